// Batched AES: many messages of uneven length, each with its own key, key
// size and mode, in one persistent launch per LDS table set, with the key
// schedules expanded on the device inside the launch.
//
// * Host plan: every message is cut into message-pure tiles of at most
//   `tile_blocks` blocks.  Tiles that need the forward tables (ECB
//   encryption, CTR either way) and tiles that need the inverse tables (ECB
//   decryption) form two queues, each sorted longest first, so that the short
//   tiles fill the end of the launch.
// * Device: each workgroup (1024 threads, one per CU) stages its table set in
//   LDS once.  Each wave then pulls tile numbers from an atomic counter until
//   the queue is empty (every wave reaches that exit; no wave waits on
//   another).  For each tile the wave expands the message key (FIPS-197
//   KeyExpansion, the key schedule the paper's section 2.1 defers to) with
//   wave-uniform table reads, so the round keys end up in SGPRs; decryption
//   keys get InvMixColumns lane-parallel.  The rounds are the single-buffer
//   kernel's (Eq. (1)); CTR tiles precompute their round-1 constants.
// * The counter reset and the persistent launches are captured once into a
//   hipGraph and replayed; the graph is re-captured when the buffers change.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "aes_device.h"
#include "aes_internal.h"

namespace aesgpu {
namespace {

using namespace dev;

struct alignas(16) DevMsg {
    uint64_t in_off;
    uint64_t out_off;
    uint64_t n_full;    // whole blocks
    uint32_t tail;      // bytes of a final partial block (CTR only)
    uint32_t key_slot;
    uint32_t nr;
    uint32_t mode;      // AESGPU_MODE_ECB / AESGPU_MODE_CTR
    uint32_t nonce[3];
    uint32_t ctr0;
    uint32_t pad[2];
};
static_assert(sizeof(DevMsg) == 64, "descriptor layout");

struct alignas(16) Tile {
    uint32_t msg;
    uint32_t n_blocks;      // blocks in this tile (the partial CTR block counts)
    uint64_t first_block;   // first block of the tile within its message
};
static_assert(sizeof(Tile) == 16, "tile layout");

struct BatchParams {
    const DevMsg *msgs;
    const Tile *tiles;
    uint32_t n_tiles;
    uint32_t *counter;
    const uint8_t *keys;   // raw key bytes, 32-byte stride
    const uint8_t *in;
    uint8_t *out;
    const uint32_t *tables;
};

// Wave-uniform reads of copy 0 of a table (every lane reads the same word, so
// the LDS broadcasts it and the compiler moves the result to an SGPR).
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

template <bool kInv>
__device__ __forceinline__ uint32_t sbox_u(const uint32_t *lds, uint32_t x) {
    // Forward set: S(x) is byte 1 of T0[x]; inverse set: byte 1 of the S word.
    const uint32_t w = kInv ? lds_at(lds, kInvSByte + (x << 7)) : lds_at(lds, x << 8);
    return (uniform(w) >> 8) & 0xFFu;
}

template <bool kInv>
__device__ __forceinline__ uint32_t sub_word_u(const uint32_t *lds, uint32_t w) {
    return sbox_u<kInv>(lds, w & 0xFFu) | (sbox_u<kInv>(lds, (w >> 8) & 0xFFu) << 8) |
           (sbox_u<kInv>(lds, (w >> 16) & 0xFFu) << 16) | (sbox_u<kInv>(lds, w >> 24) << 24);
}

// T_t[x] (or Td_t[x]) from copy 0.
__device__ __forceinline__ uint32_t table_u(const uint32_t *lds, int t, uint32_t x) {
    return uniform(lds_at(lds, uint32_t(t >> 1) * 65536u + (x << 8) + uint32_t(t & 1) * 128u));
}

// FIPS-197 KeyExpansion.  Word i of the schedule (little-endian) is computed
// in SGPRs and stored in lane i of the returned VGPR, so a whole schedule
// occupies one register; only the last nk words stay live in SGPRs for the
// recurrence.
template <bool kInv, int NR>
__device__ __forceinline__ uint32_t expand_key(const uint32_t *lds, const uint32_t *key) {
    constexpr int nk = NR - 6;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t win[8];  // win[i % nk] = word i
    uint32_t kreg = 0;
#pragma unroll
    for (int i = 0; i < nk; ++i) {
        win[i] = uniform(key[i]);
        kreg = lane == uint32_t(i) ? win[i] : kreg;
    }
    uint32_t rcon = 1;
#pragma unroll
    for (int i = nk; i < 4 * (NR + 1); ++i) {
        uint32_t t = win[(i - 1) % nk];
        if (i % nk == 0) {
            // RotWord is a right rotation of the little-endian word.
            t = sub_word_u<kInv>(lds, (t >> 8) | (t << 24)) ^ rcon;
            rcon = ((rcon << 1) ^ ((rcon >> 7) * 0x1Bu)) & 0xFFu;  // x * rcon in GF(2^8)
        } else if (nk == 8 && i % nk == 4) {
            t = sub_word_u<kInv>(lds, t);
        }
        win[i % nk] = uniform(win[i % nk] ^ t);
        kreg = lane == uint32_t(i) ? win[i % nk] : kreg;
    }
    return kreg;
}

// Equivalent inverse cipher keys from the encryption schedule (both one word
// per lane): decryption round r is encryption round NR - r, with
// InvMixColumns applied to rounds 1..NR-1.  InvMixColumns(w) is the XOR of
// Td_k[S(byte k of w)], read from the lane's own table copies.
template <int NR>
__device__ __forceinline__ uint32_t decrypt_keys(const uint32_t *lds, const Bases &b,
                                                 uint32_t enc) {
    const uint32_t i = threadIdx.x & 63u;
    const uint32_t src = i < 4 * NR + 4 ? 4 * (NR - i / 4) + (i & 3) : 0;
    const uint32_t w = __builtin_amdgcn_ds_bpermute(int(src * 4), int(enc));
    if (i < 4 || i >= 4 * NR) return w;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t x = (w >> (8 * k)) & 0xFFu;
        const uint32_t s = (lds_at(lds, (x << 7) + b.invs) >> 8) & 0xFFu;
        acc ^= lds_at(lds, __builtin_amdgcn_perm(s, b.t[k], 0x0C020400u));
    }
    return acc;
}

// Round key r as four SGPRs, read from the schedule register.
__device__ __forceinline__ void round_key(uint32_t kreg, int r, uint32_t (&k)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) k[c] = __builtin_amdgcn_readlane(kreg, 4 * r + c);
}

// One tile: NR rounds on BPL blocks per lane per step.
template <bool kInv, int NR, int BPL>
__device__ __forceinline__ void run_tile(const uint32_t *lds, const Bases &b, const BatchParams &p,
                                         const DevMsg &m, const Tile &tile) {
    const uint32_t *key = reinterpret_cast<const uint32_t *>(p.keys + 32ull * m.key_slot);
    uint32_t kreg = expand_key<kInv, NR>(lds, key);
    if constexpr (kInv) kreg = decrypt_keys<NR>(lds, b, kreg);

    const bool ctr = !kInv && m.mode == AESGPU_MODE_CTR;
    CtrConsts cc{};
    if (!kInv && ctr) {
        // Counter words 0..2 are the nonce for every block of the message.
        uint32_t k0[4], k1[4];
        round_key(kreg, 0, k0);
        round_key(kreg, 1, k1);
        uint32_t x[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) x[c] = m.nonce[c] ^ k0[c];
        cc.k03 = k0[3];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            uint32_t v = k1[c];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = (c + k) & 3;
                if (i != 3) v ^= table_u(lds, k, (x[i] >> (8 * k)) & 0xFFu);
            }
            cc.p[c] = v;
        }
    }

    const uint32_t lane = threadIdx.x & 63u;
    const uint4 *in = reinterpret_cast<const uint4 *>(p.in + m.in_off);
    uint4 *out = reinterpret_cast<uint4 *>(p.out + m.out_off);
    const uint64_t end = tile.first_block + tile.n_blocks;
    constexpr uint32_t kStep = 64u * BPL;
    for (uint64_t base = tile.first_block; base < end; base += kStep) {
        // Keep the round-key reads inside the loop: hoisting all of them would
        // need 4 * (NR + 1) SGPRs at once.
        asm volatile("" : "+v"(kreg));
        uint32_t s[BPL][4];
        uint4 d[BPL];
        uint32_t rk[4];
        round_key(kreg, 0, rk);
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            const uint64_t idx = base + uint64_t(j) * 64u + lane;
            d[j] = make_uint4(0, 0, 0, 0);
            if (idx < end && idx < m.n_full) d[j] = in[idx];
            if (ctr) {
                const uint32_t w3 = __builtin_amdgcn_perm(m.ctr0 + uint32_t(idx),
                                                          m.ctr0 + uint32_t(idx), 0x00010203u) ^
                                    cc.k03;
                s[j][0] = cc.p[0] ^ tlook<3>(lds, w3, b.t[3]);
                s[j][1] = cc.p[1] ^ tlook<2>(lds, w3, b.t[2]);
                s[j][2] = cc.p[2] ^ tlook<1>(lds, w3, b.t[1]);
                s[j][3] = cc.p[3] ^ tlook<0>(lds, w3, b.t[0]);
            } else {
                s[j][0] = d[j].x ^ rk[0];
                s[j][1] = d[j].y ^ rk[1];
                s[j][2] = d[j].z ^ rk[2];
                s[j][3] = d[j].w ^ rk[3];
            }
        }
        if (!ctr) {
            round_key(kreg, 1, rk);
#pragma unroll
            for (int j = 0; j < BPL; ++j) mid_round<kInv>(lds, b, s[j], rk);
        }
#pragma unroll
        for (int r = 2; r < NR; ++r) {
            round_key(kreg, r, rk);
#pragma unroll
            for (int j = 0; j < BPL; ++j) mid_round<kInv>(lds, b, s[j], rk);
        }
        round_key(kreg, NR, rk);
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            if constexpr (kInv)
                last_round_inv(lds, b, s[j], rk);
            else
                last_round_fwd(lds, b, s[j], rk);
        }
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            const uint64_t idx = base + uint64_t(j) * 64u + lane;
            if (idx >= end) continue;
            uint4 o = make_uint4(s[j][0], s[j][1], s[j][2], s[j][3]);
            if (ctr) {
                o.x ^= d[j].x;
                o.y ^= d[j].y;
                o.z ^= d[j].z;
                o.w ^= d[j].w;
            }
            if (idx < m.n_full) {
                out[idx] = o;
            } else if (ctr && idx == m.n_full && m.tail) {
                const uint8_t *src = reinterpret_cast<const uint8_t *>(in + m.n_full);
                uint8_t *dst = reinterpret_cast<uint8_t *>(out + m.n_full);
                const uint32_t ks[4] = {s[j][0], s[j][1], s[j][2], s[j][3]};
                for (uint32_t q = 0; q < m.tail; ++q)
                    dst[q] = src[q] ^ uint8_t(ks[q >> 2] >> (8 * (q & 3)));
            }
        }
    }
}

template <bool kInv, int BPL>
__global__ __launch_bounds__(kWG) void batch_kernel(BatchParams p) {
    __shared__ uint32_t lds[kInv ? kFwdWords + kInvSWords : kFwdWords];
    stage_tables<kInv>(lds, p.tables);
    const Bases b = lane_bases();
    const DevMsg *__restrict__ msgs = p.msgs;
    const Tile *__restrict__ tiles = p.tiles;
    for (;;) {
        uint32_t t = 0;
        if ((threadIdx.x & 63u) == 0) t = atomicAdd(p.counter, 1u);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= p.n_tiles) break;
        const Tile tile = tiles[t];
        const DevMsg m = msgs[tile.msg];
        if (m.nr == 10)
            run_tile<kInv, 10, BPL>(lds, b, p, m, tile);
        else if (m.nr == 12)
            run_tile<kInv, 12, BPL>(lds, b, p, m, tile);
        else
            run_tile<kInv, 14, BPL>(lds, b, p, m, tile);
    }
}

__global__ void reset_counters(uint32_t *c, uint32_t n) {
    if (threadIdx.x < n) c[threadIdx.x] = 0;
}

constexpr uint32_t kDefaultBpl = 4;
constexpr uint32_t kDefaultTileBlocks = 2048;

}  // namespace
}  // namespace aesgpu

using namespace aesgpu;

struct aesgpu_batch {
    aesgpu_ctx *ctx = nullptr;
    uint32_t bpl = kDefaultBpl;
    uint32_t tile_blocks = kDefaultTileBlocks;
    bool use_graph = true;
    size_t n_msgs = 0;
    size_t n_tiles[2] = {0, 0};    // forward, inverse
    uint64_t total_bytes = 0;
    uint64_t in_end = 0, out_end = 0;
    uint32_t max_slot = 0;
    void *d_mem = nullptr;         // messages | forward tiles | inverse tiles | counters
    DevMsg *d_msgs = nullptr;
    Tile *d_tiles[2] = {nullptr, nullptr};
    uint32_t *d_counters = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *cap_keys = nullptr, *cap_in = nullptr;
    void *cap_out = nullptr;
};

namespace {

uint32_t le32(const uint8_t *p) {
    return uint32_t(p[0]) | (uint32_t(p[1]) << 8) | (uint32_t(p[2]) << 16) | (uint32_t(p[3]) << 24);
}

class DeviceGuard {
  public:
    explicit DeviceGuard(int device) {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        ok_ = prev_ == device || hipSetDevice(device) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev_ >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

  private:
    int prev_ = -1;
    bool ok_ = false;
};

void release_graph(aesgpu_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

template <int BPL>
int enqueue_t(aesgpu_batch *b, const uint8_t *keys, const void *in, void *out, hipStream_t s) {
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, b->d_counters, 2u);
    for (int set = 0; set < 2; ++set) {
        if (!b->n_tiles[set]) continue;
        BatchParams p{b->d_msgs, b->d_tiles[set], uint32_t(b->n_tiles[set]), b->d_counters + set,
                      keys, static_cast<const uint8_t *>(in), static_cast<uint8_t *>(out),
                      b->ctx->d_tables};
        const uint32_t grid = uint32_t(std::min<size_t>(b->ctx->n_cu, b->n_tiles[set]));
        if (set == 0)
            hipLaunchKernelGGL((batch_kernel<false, BPL>), dim3(grid), dim3(kWG), 0, s, p);
        else
            hipLaunchKernelGGL((batch_kernel<true, BPL>), dim3(grid), dim3(kWG), 0, s, p);
    }
    return hipGetLastError() == hipSuccess ? AESGPU_OK : AESGPU_EHIP;
}

int enqueue(aesgpu_batch *b, const uint8_t *keys, const void *in, void *out, hipStream_t s) {
    return b->bpl == 2 ? enqueue_t<2>(b, keys, in, out, s) : enqueue_t<4>(b, keys, in, out, s);
}

}  // namespace

extern "C" {

int aesgpu_batch_plan(aesgpu_ctx *ctx, const aesgpu_msg *msgs, size_t m,
                      const aesgpu_batch_config *cfg, aesgpu_batch **out) {
    if (!out) return AESGPU_EINVAL;
    *out = nullptr;
    if (!ctx || (m > 0 && !msgs)) return AESGPU_EINVAL;
    if (m > 0xFFFFFFFFull) return AESGPU_EINVAL;
    uint32_t bpl = kDefaultBpl, tile_blocks = kDefaultTileBlocks;
    bool use_graph = true;
    if (cfg) {
        if (cfg->blocks_per_lane) bpl = cfg->blocks_per_lane;
        if (cfg->tile_blocks) tile_blocks = cfg->tile_blocks;
        use_graph = !(cfg->flags & AESGPU_BATCH_NO_GRAPH);
    }
    if (bpl != 2 && bpl != 4) return AESGPU_EINVAL;
    if (tile_blocks % (64u * bpl) != 0 || tile_blocks > (1u << 24)) return AESGPU_EINVAL;

    std::vector<DevMsg> dm(m);
    std::vector<Tile> tiles[2];
    uint64_t total = 0, in_end = 0, out_end = 0;
    uint32_t max_slot = 0;
    for (size_t i = 0; i < m; ++i) {
        const aesgpu_msg &x = msgs[i];
        if (x.key_bits != 128 && x.key_bits != 192 && x.key_bits != 256) return AESGPU_EKEYLEN;
        if (x.mode != AESGPU_MODE_ECB && x.mode != AESGPU_MODE_CTR) return AESGPU_EINVAL;
        if (x.dir != AESGPU_DIR_ENCRYPT && x.dir != AESGPU_DIR_DECRYPT) return AESGPU_EINVAL;
        if ((x.in_off & 15u) || (x.out_off & 15u)) return AESGPU_EALIGN;
        if (x.mode == AESGPU_MODE_ECB && (x.n_bytes & 15u)) return AESGPU_EINVAL;
        if (x.n_bytes > (UINT64_MAX >> 1) || x.in_off > UINT64_MAX - x.n_bytes ||
            x.out_off > UINT64_MAX - x.n_bytes)
            return AESGPU_EINVAL;
        const uint64_t n_blocks = (x.n_bytes + 15) / 16;
        if (x.mode == AESGPU_MODE_CTR && n_blocks && uint64_t(x.ctr0) + n_blocks - 1 > 0xFFFFFFFFull)
            return AESGPU_ECTR_OVERFLOW;
        DevMsg &d = dm[i];
        d = DevMsg{};
        d.in_off = x.in_off;
        d.out_off = x.out_off;
        d.n_full = x.n_bytes / 16;
        d.tail = uint32_t(x.n_bytes % 16);
        d.key_slot = x.key_slot;
        d.nr = x.key_bits / 32 + 6;
        d.mode = x.mode;
        for (int c = 0; c < 3; ++c) d.nonce[c] = le32(x.nonce + 4 * c);
        d.ctr0 = x.ctr0;
        total += x.n_bytes;
        if (x.n_bytes) {
            in_end = std::max(in_end, x.in_off + x.n_bytes);
            out_end = std::max(out_end, x.out_off + x.n_bytes);
            max_slot = std::max(max_slot, x.key_slot);
        }
        const int set = (x.mode == AESGPU_MODE_ECB && x.dir == AESGPU_DIR_DECRYPT) ? 1 : 0;
        for (uint64_t f = 0; f < n_blocks; f += tile_blocks) {
            const uint64_t n = std::min<uint64_t>(tile_blocks, n_blocks - f);
            tiles[set].push_back(Tile{uint32_t(i), uint32_t(n), f});
        }
    }
    for (auto &t : tiles)
        std::stable_sort(t.begin(), t.end(),
                         [](const Tile &a, const Tile &b) { return a.n_blocks > b.n_blocks; });

    aesgpu_batch *b = new (std::nothrow) aesgpu_batch;
    if (!b) return AESGPU_ENOMEM;
    b->ctx = ctx;
    b->bpl = bpl;
    b->tile_blocks = tile_blocks;
    b->use_graph = use_graph;
    b->n_msgs = m;
    b->n_tiles[0] = tiles[0].size();
    b->n_tiles[1] = tiles[1].size();
    b->total_bytes = total;
    b->in_end = in_end;
    b->out_end = out_end;
    b->max_slot = max_slot;

    DeviceGuard g(ctx->device);
    if (!g.ok()) {
        delete b;
        return AESGPU_EHIP;
    }
    const size_t msg_bytes = m * sizeof(DevMsg);
    const size_t t0 = tiles[0].size() * sizeof(Tile), t1 = tiles[1].size() * sizeof(Tile);
    const size_t bytes = msg_bytes + t0 + t1 + 64;
    if (hipMalloc(&b->d_mem, bytes) != hipSuccess) {
        delete b;
        return AESGPU_ENOMEM;
    }
    char *base = static_cast<char *>(b->d_mem);
    b->d_msgs = reinterpret_cast<DevMsg *>(base);
    b->d_tiles[0] = reinterpret_cast<Tile *>(base + msg_bytes);
    b->d_tiles[1] = reinterpret_cast<Tile *>(base + msg_bytes + t0);
    b->d_counters = reinterpret_cast<uint32_t *>(base + msg_bytes + t0 + t1);
    bool ok = true;
    if (msg_bytes) ok &= hipMemcpy(b->d_msgs, dm.data(), msg_bytes, hipMemcpyHostToDevice) == hipSuccess;
    if (t0) ok &= hipMemcpy(b->d_tiles[0], tiles[0].data(), t0, hipMemcpyHostToDevice) == hipSuccess;
    if (t1) ok &= hipMemcpy(b->d_tiles[1], tiles[1].data(), t1, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        aesgpu_batch_free(b);
        return AESGPU_EHIP;
    }
    *out = b;
    return AESGPU_OK;
}

int aesgpu_batch_run(aesgpu_batch *b, const uint8_t *d_keys, size_t n_key_slots, const void *d_in,
                     size_t in_bytes, void *d_out, size_t out_bytes, aesgpu_stream_t stream) {
    if (!b) return AESGPU_EINVAL;
    if (b->n_tiles[0] + b->n_tiles[1] == 0) return AESGPU_OK;
    if (!d_keys || !d_in || !d_out) return AESGPU_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_keys) | reinterpret_cast<uintptr_t>(d_in) |
         reinterpret_cast<uintptr_t>(d_out)) & 15u)
        return AESGPU_EALIGN;
    if (uint64_t(b->max_slot) >= n_key_slots) return AESGPU_EINVAL;
    if (b->in_end > in_bytes || b->out_end > out_bytes) return AESGPU_EINVAL;
    const uintptr_t i0 = reinterpret_cast<uintptr_t>(d_in), o0 = reinterpret_cast<uintptr_t>(d_out);
    if (i0 != o0 && i0 < o0 + out_bytes && o0 < i0 + in_bytes) return AESGPU_EINVAL;
    DeviceGuard g(b->ctx->device);
    if (!g.ok()) return AESGPU_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!b->use_graph) return enqueue(b, d_keys, d_in, d_out, s);
    if (!b->exec || b->cap_keys != d_keys || b->cap_in != d_in || b->cap_out != d_out) {
        release_graph(b);
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return AESGPU_EHIP;
        const int st = enqueue(b, d_keys, d_in, d_out, b->cap_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
        if (st != AESGPU_OK || e != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return AESGPU_EHIP;
        }
        b->graph = graph;
        if (hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            release_graph(b);
            return AESGPU_EHIP;
        }
        b->cap_keys = d_keys;
        b->cap_in = d_in;
        b->cap_out = d_out;
    }
    return hipGraphLaunch(b->exec, s) == hipSuccess ? AESGPU_OK : AESGPU_EHIP;
}

int aesgpu_batch_info(const aesgpu_batch *b, aesgpu_batch_stats *out) {
    if (!b || !out) return AESGPU_EINVAL;
    out->n_msgs = b->n_msgs;
    out->n_tiles_forward = b->n_tiles[0];
    out->n_tiles_inverse = b->n_tiles[1];
    out->total_bytes = b->total_bytes;
    out->in_bytes_needed = b->in_end;
    out->out_bytes_needed = b->out_end;
    out->blocks_per_lane = b->bpl;
    out->tile_blocks = b->tile_blocks;
    out->launches = (b->n_tiles[0] ? 1u : 0u) + (b->n_tiles[1] ? 1u : 0u);
    return AESGPU_OK;
}

void aesgpu_batch_free(aesgpu_batch *b) {
    if (!b) return;
    {
        DeviceGuard g(b->ctx->device);
        release_graph(b);
        if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
        if (b->d_mem) (void)hipFree(b->d_mem);
    }
    delete b;
}

}  // extern "C"
