// Host-side checks of the library's CPU logic, for sanitizer builds that run
// without a GPU (tests/test_host_sanitizers.py builds this file with
// AddressSanitizer + UndefinedBehaviorSanitizer, and with ThreadSanitizer).
//
// Covered: key expansion (all lengths), argument validation of the buffer
// calls (every path that returns before a HIP call), the batch planner
// (build_tiles: random batches checked for exact coverage, tile bounds,
// queue order and CBC groups; every error class), the allocation-free batch
// call's host staging (up to the point where it needs a GPU), the server's
// range allocator (random alloc / release against its invariants, and one
// arena shared by several threads under a lock, as the server uses it), and
// the pipeline's host copy pool (parallel copies checked byte for byte, many
// pools at once from several threads).
//
// This file includes aes_pipeline.cpp to reach its file-local CopyPool; the
// other library sources are linked as objects compiled for the host only.
//
// Usage: host_checks asan|tsan      (exit status 0 and "host checks ok")
#include "aes_pipeline.cpp"

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <thread>

#include "aes_batch.h"

namespace {

std::atomic<int> g_failures{0};
std::atomic<long> g_checks{0};

#define EXPECT(cond)                                                          \
    do {                                                                      \
        ++g_checks;                                                           \
        if (!(cond)) {                                                        \
            std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++g_failures;                                                     \
        }                                                                     \
    } while (0)

// ---- key expansion --------------------------------------------------------

void check_key_expansion() {
    uint8_t key[64];
    for (int i = 0; i < 64; ++i) key[i] = uint8_t(i * 29 + 7);
    for (size_t n = 0; n <= 40; ++n) {
        aesgpu_key k;
        const int st = aesgpu_expand_key(key, n, &k);
        if (n == 16 || n == 24 || n == 32) {
            EXPECT(st == AESGPU_OK);
            EXPECT(k.key_bits == 8 * n && k.nr == n / 4 + 6);
            EXPECT(key_ok(&k));
            // The first Nk words are the key itself (little-endian words).
            for (size_t w = 0; w < n / 4; ++w) EXPECT(k.enc[w] == le32(key + 4 * w));
            // Equivalent inverse cipher: dec[0] = enc round Nr, dec[Nr] = enc round 0.
            for (int c = 0; c < 4; ++c) {
                EXPECT(k.dec[c] == k.enc[4 * k.nr + c]);
                EXPECT(k.dec[4 * k.nr + c] == k.enc[c]);
            }
        } else {
            EXPECT(st == AESGPU_EKEYLEN);
        }
    }
    aesgpu_key k;
    EXPECT(aesgpu_expand_key(nullptr, 16, &k) == AESGPU_EINVAL);
    EXPECT(aesgpu_expand_key(key, 16, nullptr) == AESGPU_EINVAL);
}

// ---- argument validation (paths that end before any HIP call) -------------

void check_validation() {
    aesgpu_ctx fake{0, 256, nullptr};
    uint8_t key[16] = {1, 2, 3};
    aesgpu_key k;
    EXPECT(aesgpu_expand_key(key, 16, &k) == AESGPU_OK);
    // Addresses that are never dereferenced on the host.
    void *a = reinterpret_cast<void *>(uintptr_t(1) << 32);
    void *b = reinterpret_cast<void *>((uintptr_t(1) << 32) + (uintptr_t(1) << 24));
    void *odd = reinterpret_cast<void *>((uintptr_t(1) << 32) + 8);
    const uint8_t nonce[12] = {0};
    const uint8_t iv[16] = {0};
    EXPECT(aesgpu_ecb_encrypt(nullptr, &k, a, b, 4, nullptr) == AESGPU_EINVAL);
    EXPECT(aesgpu_ecb_encrypt(&fake, nullptr, a, b, 4, nullptr) == AESGPU_EINVAL);
    EXPECT(aesgpu_ecb_encrypt(&fake, &k, a, b, 0, nullptr) == AESGPU_OK);
    EXPECT(aesgpu_ecb_encrypt(&fake, &k, odd, b, 4, nullptr) == AESGPU_EALIGN);
    EXPECT(aesgpu_ecb_decrypt(&fake, &k, a, odd, 4, nullptr) == AESGPU_EALIGN);
    EXPECT(aesgpu_ecb_decrypt(&fake, &k, nullptr, b, 4, nullptr) == AESGPU_EINVAL);
    // Partial overlap (16 bytes apart, 4 blocks long).
    void *a16 = reinterpret_cast<void *>((uintptr_t(1) << 32) + 16);
    EXPECT(aesgpu_ecb_encrypt(&fake, &k, a, a16, 4, nullptr) == AESGPU_EINVAL);
    EXPECT(aesgpu_ctr_xcrypt(&fake, &k, nonce, 0xFFFFFFFFu, a, b, 33, nullptr) ==
           AESGPU_ECTR_OVERFLOW);
    EXPECT(aesgpu_ctr_xcrypt(&fake, &k, nullptr, 1, a, b, 33, nullptr) == AESGPU_EINVAL);
    EXPECT(aesgpu_cbc_decrypt(&fake, &k, iv, a, a, 4, nullptr) == AESGPU_EINVAL);  // in place
    EXPECT(aesgpu_cbc_decrypt(&fake, &k, nullptr, a, b, 4, nullptr) == AESGPU_EINVAL);
    aesgpu_key bad = k;
    bad.nr = 11;
    EXPECT(aesgpu_ecb_encrypt(&fake, &bad, a, b, 4, nullptr) == AESGPU_EINVAL);
    EXPECT(std::string(aesgpu_strerror(AESGPU_ESCRATCH)).size() > 0);
    EXPECT(std::string(aesgpu_strerror(-1000)).size() > 0);
}

// ---- batch planner ---------------------------------------------------------

std::vector<aesgpu_msg> random_batch(std::mt19937_64 &rng, size_t m, uint64_t max_bytes) {
    std::vector<aesgpu_msg> v(m);
    uint64_t in = 0, out = uint64_t(1) << 40;
    for (size_t i = 0; i < m; ++i) {
        aesgpu_msg &x = v[i];
        x = aesgpu_msg{};
        x.mode = uint8_t(rng() % 3);
        x.dir = uint8_t(rng() % 2);
        x.key_bits = uint16_t(128 + 64 * (rng() % 3));
        x.key_slot = uint32_t(rng() % 50);
        uint64_t n = rng() % (max_bytes + 1);
        if (x.mode != AESGPU_MODE_CTR) n &= ~uint64_t(15);
        if (rng() % 17 == 0) n = 0;
        x.n_bytes = n;
        x.ctr0 = uint32_t(rng() % (1u << 30));
        for (int c = 0; c < 12; ++c) x.nonce[c] = uint8_t(rng());
        x.in_off = in;
        x.out_off = out;
        in += (n + 15) / 16 * 16 + 16 * (rng() % 3);
        out += (n + 15) / 16 * 16;
    }
    return v;
}

void check_plan(const std::vector<aesgpu_msg> &msgs, uint32_t tile_blocks) {
    std::vector<DevMsg> dm;
    std::vector<Tile> tiles[2];
    std::vector<uint32_t> cbc_list;
    std::vector<Tile> cbc_groups;
    BatchTotals tot;
    const size_t m = msgs.size();
    EXPECT(build_tiles(msgs.data(), m, tile_blocks, dm, tiles, cbc_list, cbc_groups, tot) ==
           AESGPU_OK);
    EXPECT(dm.size() == m);
    // Every block of every non-CBC-encrypt message is in exactly one tile of
    // the right queue; tiles stay within tile_blocks; queues longest first.
    std::vector<std::vector<std::pair<uint64_t, uint64_t>>> cover(m);
    uint64_t blocks[2] = {0, 0};
    for (int set = 0; set < 2; ++set) {
        for (size_t t = 0; t < tiles[set].size(); ++t) {
            const Tile &x = tiles[set][t];
            EXPECT(x.msg < m);
            if (x.msg >= m) continue;
            EXPECT(x.n_blocks >= 1 && x.n_blocks <= tile_blocks);
            if (t) EXPECT(tiles[set][t - 1].n_blocks >= x.n_blocks);
            const aesgpu_msg &g = msgs[x.msg];
            const bool inverse = g.mode != AESGPU_MODE_CTR && g.dir == AESGPU_DIR_DECRYPT;
            EXPECT(set == (inverse ? 1 : 0));
            EXPECT(!(g.mode == AESGPU_MODE_CBC && g.dir == AESGPU_DIR_ENCRYPT));
            cover[x.msg].push_back({x.first_block, x.first_block + x.n_blocks});
            blocks[set] += x.n_blocks;
            // CTR tiles after a message's first start at a counter that is a
            // multiple of 256 when the tile size is one.
            if (g.mode == AESGPU_MODE_CTR && tile_blocks % 256 == 0 && x.first_block > 0)
                EXPECT((uint64_t(g.ctr0) + x.first_block) % 256 == 0);
        }
    }
    EXPECT(blocks[0] == tot.blocks[0] && blocks[1] == tot.blocks[1]);
    std::vector<int> in_cbc(m, 0);
    for (uint32_t i : cbc_list) {
        EXPECT(i < m);
        if (i < m) ++in_cbc[i];
    }
    uint64_t total = 0;
    for (size_t i = 0; i < m; ++i) {
        const aesgpu_msg &g = msgs[i];
        total += g.n_bytes;
        const uint64_t nb = (g.n_bytes + 15) / 16;
        EXPECT(dm[i].n_full == g.n_bytes / 16 && dm[i].tail == g.n_bytes % 16);
        EXPECT(dm[i].nr == uint32_t(g.key_bits / 32 + 6));
        if (g.mode == AESGPU_MODE_CBC && g.dir == AESGPU_DIR_ENCRYPT) {
            EXPECT(cover[i].empty());
            EXPECT(in_cbc[i] == (nb ? 1 : 0));
            continue;
        }
        EXPECT(in_cbc[i] == 0);
        auto &c = cover[i];
        std::sort(c.begin(), c.end());
        uint64_t at = 0;
        for (auto &r : c) {
            EXPECT(r.first == at);
            at = r.second;
        }
        EXPECT(at == nb);
    }
    EXPECT(total == tot.total);
    // CBC-encrypt groups: at most 16 messages of one key size each, the
    // group's longest block count first in the group, groups longest first.
    size_t listed = 0;
    for (size_t gi = 0; gi < cbc_groups.size(); ++gi) {
        const Tile &gr = cbc_groups[gi];
        EXPECT(gr.n_blocks >= 1 && gr.n_blocks <= kCbcGroupMsgs);
        EXPECT(size_t(gr.msg) + gr.n_blocks <= cbc_list.size());
        if (size_t(gr.msg) + gr.n_blocks > cbc_list.size()) continue;
        const uint16_t bits = msgs[cbc_list[gr.msg]].key_bits;
        for (uint32_t j = 0; j < gr.n_blocks; ++j) {
            const uint32_t mi = cbc_list[gr.msg + j];
            EXPECT(msgs[mi].key_bits == bits);
            EXPECT(dm[mi].n_full <= gr.first_block);
        }
        EXPECT(dm[cbc_list[gr.msg]].n_full == gr.first_block);
        if (gi) EXPECT(cbc_groups[gi - 1].first_block >= gr.first_block);
        listed += gr.n_blocks;
    }
    EXPECT(listed == cbc_list.size());
}

void check_planner() {
    std::mt19937_64 rng(42);
    for (int round = 0; round < 60; ++round) {
        const size_t m = 1 + rng() % 700;
        const uint64_t max_bytes = round % 3 == 0 ? 64 : round % 3 == 1 ? 20000 : 1 << 20;
        const uint32_t tile = (round % 4 == 0) ? 64 : (round % 4 == 1) ? 256 : 8192;
        check_plan(random_batch(rng, m, max_bytes), tile);
    }
    // Error classes, each on a message in the middle of a valid batch.
    std::vector<DevMsg> dm;
    std::vector<Tile> tiles[2];
    std::vector<uint32_t> cl;
    std::vector<Tile> cg;
    BatchTotals tot;
    auto with = [&](auto edit) {
        std::vector<aesgpu_msg> v = random_batch(rng, 9, 4096);
        v[4].mode = AESGPU_MODE_ECB;
        v[4].n_bytes = 64;
        edit(v[4]);
        return build_tiles(v.data(), v.size(), 256, dm, tiles, cl, cg, tot);
    };
    EXPECT(with([](aesgpu_msg &x) { x.key_bits = 130; }) == AESGPU_EKEYLEN);
    EXPECT(with([](aesgpu_msg &x) { x.mode = 3; }) == AESGPU_EINVAL);
    EXPECT(with([](aesgpu_msg &x) { x.dir = 2; }) == AESGPU_EINVAL);
    EXPECT(with([](aesgpu_msg &x) { x.in_off += 8; }) == AESGPU_EALIGN);
    EXPECT(with([](aesgpu_msg &x) { x.out_off += 4; }) == AESGPU_EALIGN);
    EXPECT(with([](aesgpu_msg &x) { x.n_bytes = 33; }) == AESGPU_EINVAL);
    EXPECT(with([](aesgpu_msg &x) { x.n_bytes = UINT64_MAX - 15; }) == AESGPU_EINVAL);
    EXPECT(with([](aesgpu_msg &x) {
               x.mode = AESGPU_MODE_CTR;
               x.ctr0 = 0xFFFFFFFFu;
               x.n_bytes = 17;
           }) == AESGPU_ECTR_OVERFLOW);
}

// The allocation-free batch call up to the point where it needs a GPU: the
// planner, the size check and the host staging run; with no GPU the call
// then fails with EHIP.  A batch past the scratch fails with ESCRATCH.
void check_noalloc_host_path(bool gpu_calls) {
    aesgpu_ctx fake{0, 256, nullptr};
    std::mt19937_64 rng(7);
    void *keys = reinterpret_cast<void *>(uintptr_t(1) << 36);
    void *in = reinterpret_cast<void *>(uintptr_t(1) << 37);
    void *out = reinterpret_cast<void *>(uintptr_t(1) << 38);
    std::vector<aesgpu_msg> big(AESGPU_NOALLOC_SCRATCH_BYTES / 64 + 1);
    for (size_t i = 0; i < big.size(); ++i) {
        big[i] = aesgpu_msg{};
        big[i].key_bits = 128;
        big[i].n_bytes = 16;
        big[i].in_off = big[i].out_off = 16 * i;
    }
    EXPECT(aesgpu_batch_run_noalloc(&fake, big.data(), big.size(), nullptr,
                                    static_cast<const uint8_t *>(keys), 1, in, 16 * big.size(),
                                    out, 16 * big.size(), nullptr) == AESGPU_ESCRATCH);
    EXPECT(aesgpu_batch_run_noalloc(nullptr, big.data(), 1, nullptr,
                                    static_cast<const uint8_t *>(keys), 1, in, 16, out, 16,
                                    nullptr) == AESGPU_EINVAL);
    aesgpu_batch_config cfg{3, 0, 0};
    EXPECT(aesgpu_batch_run_noalloc(&fake, big.data(), 1, &cfg,
                                    static_cast<const uint8_t *>(keys), 1, in, 16, out, 16,
                                    nullptr) == AESGPU_EINVAL);
    // Key slots and buffer sizes are checked against the batch.
    EXPECT(aesgpu_batch_run_noalloc(&fake, big.data(), 4, nullptr,
                                    static_cast<const uint8_t *>(keys), 1, in, 32, out, 64,
                                    nullptr) == AESGPU_EINVAL);
    if (!gpu_calls) return;
    for (int round = 0; round < 5; ++round) {
        std::vector<aesgpu_msg> v = random_batch(rng, 1 + rng() % 300, 1 << 16);
        uint64_t in_end = 0, out_end = 0;
        for (auto &x : v) {
            in_end = std::max(in_end, x.in_off + x.n_bytes);
            out_end = std::max(out_end, x.out_off + x.n_bytes);
        }
        const int st = aesgpu_batch_run_noalloc(&fake, v.data(), v.size(), nullptr,
                                                static_cast<const uint8_t *>(keys), 50, in,
                                                in_end, out, out_end, nullptr);
        EXPECT(st == AESGPU_EHIP || st == AESGPU_OK);
    }
}

// ---- range allocator ---------------------------------------------------------

void arena_random(aesgpu_arena *a, uint64_t cap, uint64_t granule, std::mt19937_64 &rng,
                  int ops, std::mutex *mu) {
    std::vector<std::pair<uint64_t, uint64_t>> live;
    for (int i = 0; i < ops; ++i) {
        if (live.empty() || rng() % 3 != 0) {
            const uint64_t n = 1 + rng() % (cap / 16);
            uint64_t off = 0;
            int st;
            {
                std::unique_lock<std::mutex> lk;
                if (mu) lk = std::unique_lock<std::mutex>(*mu);
                st = aesgpu_arena_alloc(a, n, &off);
            }
            if (st == AESGPU_OK) {
                EXPECT(off % granule == 0 && off + n <= cap);
                live.push_back({off, n});
            } else {
                EXPECT(st == AESGPU_EAGAIN);
            }
        } else {
            const size_t j = rng() % live.size();
            std::unique_lock<std::mutex> lk;
            if (mu) lk = std::unique_lock<std::mutex>(*mu);
            EXPECT(aesgpu_arena_release(a, live[j].first, live[j].second) == AESGPU_OK);
            // A second release of the same range is refused.
            EXPECT(aesgpu_arena_release(a, live[j].first, live[j].second) == AESGPU_EINVAL);
            live.erase(live.begin() + long(j));
        }
        if (!mu && i % 64 == 0) {
            // Live ranges never overlap; used bytes add up.
            std::vector<std::pair<uint64_t, uint64_t>> s = live;
            std::sort(s.begin(), s.end());
            uint64_t used_model = 0;
            for (size_t q = 0; q < s.size(); ++q) {
                const uint64_t len = (s[q].second + granule - 1) / granule * granule;
                used_model += len;
                if (q + 1 < s.size()) EXPECT(s[q].first + len <= s[q + 1].first);
            }
            uint64_t used = 0, largest = 0, high = 0;
            EXPECT(aesgpu_arena_query(a, &used, &largest, &high) == AESGPU_OK);
            EXPECT(used == used_model && largest <= cap - used && high >= used);
        }
    }
    std::unique_lock<std::mutex> lk;
    if (mu) lk = std::unique_lock<std::mutex>(*mu);
    for (auto &r : live) EXPECT(aesgpu_arena_release(a, r.first, r.second) == AESGPU_OK);
}

void check_arena(bool threaded) {
    const uint64_t cap = uint64_t(1) << 26, granule = 256;
    aesgpu_arena *a = nullptr;
    EXPECT(aesgpu_arena_create(cap, granule, &a) == AESGPU_OK && a);
    if (!a) return;
    if (!threaded) {
        std::mt19937_64 rng(3);
        arena_random(a, cap, granule, rng, 40000, nullptr);
    } else {
        // One arena, several threads, one lock: the way the server's
        // dispatcher and callers share it.
        std::mutex mu;
        std::vector<std::thread> ts;
        for (int t = 0; t < 4; ++t)
            ts.emplace_back([&, t] {
                std::mt19937_64 rng(100 + t);
                arena_random(a, cap, granule, rng, 5000, &mu);
            });
        for (auto &t : ts) t.join();
    }
    uint64_t used = 1, largest = 0, high = 0;
    EXPECT(aesgpu_arena_query(a, &used, &largest, &high) == AESGPU_OK);
    EXPECT(used == 0 && largest == cap);
    aesgpu_arena_destroy(a);
    EXPECT(aesgpu_arena_create(100, 256, &a) == AESGPU_EINVAL);
    EXPECT(aesgpu_arena_create(1024, 100, &a) == AESGPU_EINVAL);
}

// ---- host copy pool ------------------------------------------------------------

void pool_copies(CopyPool &pool, std::mt19937_64 &rng, int n) {
    std::vector<uint8_t> src(9 << 20), dst(9 << 20);
    for (size_t i = 0; i < src.size(); ++i) src[i] = uint8_t(rng());
    for (int r = 0; r < n; ++r) {
        const size_t len = (r % 3 == 0) ? rng() % 4096 : rng() % (8 << 20);
        const size_t so = rng() % (src.size() - len + 1), doff = rng() % (dst.size() - len + 1);
        std::fill(dst.begin(), dst.end(), uint8_t(0xA5));
        pool.copy(dst.data() + doff, src.data() + so, len);
        EXPECT(std::memcmp(dst.data() + doff, src.data() + so, len) == 0);
        EXPECT(doff == 0 || dst[doff - 1] == 0xA5);
        EXPECT(doff + len == dst.size() || dst[doff + len] == 0xA5);
    }
}

void check_copy_pool(bool threaded) {
    if (!threaded) {
        CopyPool pool;
        std::mt19937_64 rng(11);
        pool_copies(pool, rng, 60);
        return;
    }
    // Several pools, each used by its own thread (a pool serves one copy at
    // a time), created and destroyed repeatedly.
    std::vector<std::thread> ts;
    for (int t = 0; t < 3; ++t)
        ts.emplace_back([t] {
            std::mt19937_64 rng(20 + t);
            for (int rep = 0; rep < 3; ++rep) {
                CopyPool pool;
                pool_copies(pool, rng, 12);
            }
        });
    for (auto &t : ts) t.join();
}

}  // namespace

int main(int argc, char **argv) {
    const std::string mode = argc > 1 ? argv[1] : "asan";
    if (mode == "asan") {
        check_key_expansion();
        check_validation();
        check_planner();
        check_noalloc_host_path(true);
        check_arena(false);
        check_copy_pool(false);
    } else if (mode == "tsan") {
        check_noalloc_host_path(false);
        check_arena(true);
        check_copy_pool(true);
    } else {
        std::fprintf(stderr, "usage: host_checks asan|tsan\n");
        return 2;
    }
    if (g_failures) {
        std::fprintf(stderr, "%d host checks failed\n", g_failures.load());
        return 1;
    }
    std::printf("host checks ok (%s): %ld checks\n", mode.c_str(), g_checks.load());
    return 0;
}
