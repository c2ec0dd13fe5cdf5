// Batched AES: many messages of uneven length, each with its own key, key
// size and mode, in one persistent launch per LDS table set, with the key
// schedules expanded on the device inside the launch.
//
// * Host plan: every message is cut into message-pure tiles of at most
//   `tile_blocks` blocks.  Tiles that need the forward tables (ECB
//   encryption, CTR either way) and tiles that need the inverse tables (ECB
//   and CBC decryption) form two queues, each sorted longest first, so that
//   the short tiles fill the end of the launch.  CBC encryption is sequential
//   within a message, so CBC-encrypt messages form groups of up to 16 of one
//   key size, four lanes per message (one state column each), run by a
//   launch of their own (its round keys live in registers, which the
//   block-parallel kernel cannot spare).
// * Device: each workgroup (1024 threads, one per CU) stages its table set in
//   LDS once.  Each wave then pulls tile numbers from an atomic counter until
//   the queue is empty (every wave reaches that exit; no wave waits on
//   another).  For each tile the wave expands the message key (FIPS-197
//   KeyExpansion, the key schedule the paper's section 2.1 defers to) with
//   wave-uniform table reads into one register, word i in lane i;
//   decryption keys get InvMixColumns lane-parallel.  The rounds are the
//   single-buffer kernel's (Eq. (1)); in whole steps the middle rounds run
//   as one straight sequence shared by the three key sizes, their round keys
//   given to every lane by DPP row broadcasts.  CTR tiles precompute their
//   round-1 constants.
// * The persistent launches are captured once into a hipGraph and replayed
//   (the kernel leaves its queue counters at zero); the graph is re-captured
//   when the buffers change.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "aes_device.h"
#include "aes_batch.h"
#include "aes_internal.h"

namespace aesgpu {
namespace {

using namespace dev;

struct BatchParams {
    const DevMsg *msgs;
    const Tile *tiles[2];   // forward-set and inverse-set queues
    uint32_t n_tiles[2];
    uint32_t *counters;     // dynamic pulls of each queue, then one flag word per workgroup
    uint32_t n_wg_forward_first;  // workgroups that start on the forward queue
    uint32_t n_static[2];   // tiles handed out statically (one per wave of the starting WGs)
    uint32_t pull[2];       // consecutive tiles a wave takes per pull of a queue
    const uint8_t *keys;    // raw key bytes, 32-byte stride (device expansion)
    const uint32_t *sched;  // or resident schedules, kSchedWords per key slot
    const uint8_t *in;
    uint8_t *out;
    const uint32_t *tables;
    const uint32_t *cbc_list;  // message indices of the CBC-encryption groups
    uint4 *cbc_dummy;          // 16 bytes nobody reads (stores with nothing to store)
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
    // The lane index is re-read here: otherwise the compiler keeps the 60
    // lane comparisons below as masks through the whole launch.
    uint32_t lane = threadIdx.x & 63u;
    asm volatile("" : "+v"(lane));
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
    // The lane index is re-read here, so that the lane-dependent values below
    // are not kept in registers through the whole launch.
    uint32_t i = threadIdx.x & 63u;
    asm volatile("" : "+v"(i));
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

// Round key r (wave-uniform, possibly a run-time value) as four SGPRs, read
// from the schedule register.
__device__ __forceinline__ void round_key(uint32_t kreg, uint32_t r, uint32_t (&k)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) k[c] = __builtin_amdgcn_readlane(kreg, int(4 * r + c));
}

// Device key expansion for the message's key size.
template <bool kInv>
__device__ __forceinline__ uint32_t schedule_of(const uint32_t *lds, const Bases &b,
                                                const uint32_t *key, uint32_t nr) {
    uint32_t kreg;
    if (nr == 10) {
        kreg = expand_key<kInv, 10>(lds, key);
        if constexpr (kInv) kreg = decrypt_keys<10>(lds, b, kreg);
    } else if (nr == 12) {
        kreg = expand_key<kInv, 12>(lds, key);
        if constexpr (kInv) kreg = decrypt_keys<12>(lds, b, kreg);
    } else {
        kreg = expand_key<kInv, 14>(lds, key);
        if constexpr (kInv) kreg = decrypt_keys<14>(lds, b, kreg);
    }
    return kreg;
}

// A descriptor read through the scalar cache, word by word.
template <class T>
__device__ __forceinline__ T load_uniform(const T *src) {
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    T v;
    const auto *w = as_const(reinterpret_cast<const uint32_t *>(src));
    uint32_t *d = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) d[i] = w[i];
    return v;
}

// Round 1 of a CTR counter block (nonce words 0..2, word 3 = BE32(ctr)),
// from the per-message constants: output word c needs one lookup, on byte
// (3 - c) of word 3; the other three terms are constants.
__device__ __forceinline__ void counter_round1(const uint32_t *lds, const Bases &b,
                                               const CtrConsts &cc, uint32_t ctr,
                                               uint32_t (&s)[4]) {
    const uint32_t w3 = bswap32(ctr) ^ cc.kvar;
    s[0] = cc.p[0] ^ tlook<3>(lds, w3, b.t[3]);
    s[1] = cc.p[1] ^ tlook<2>(lds, w3, b.t[2]);
    s[2] = cc.p[2] ^ tlook<1>(lds, w3, b.t[1]);
    s[3] = cc.p[3] ^ tlook<0>(lds, w3, b.t[0]);
}

// Block loads and stores of a tile with a cache policy: 0 (the default) for
// launches, whose start and end make memory coherent; kCoherent for the
// resident kernel, whose tiles must see inputs and publish outputs
// device-wide without L2 invalidations or write-backs (sc1: agent-coherent
// accesses).
constexpr int kCoherent = 16;

template <int kPolicy>
__device__ __forceinline__ uint4 tile_load16(rsrc_t r, uint32_t offset) {
    const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, offset, 0, kPolicy);
    return make_uint4(x[0], x[1], x[2], x[3]);
}

template <int kPolicy>
__device__ __forceinline__ void tile_store16(rsrc_t r, uint32_t offset, const uint4 &v) {
    const u32x4 x = {v.x, v.y, v.z, v.w};
    __builtin_amdgcn_raw_buffer_store_b128(x, r, offset, 0, kPolicy);
}

// k[i] = lane I0 + i of x's row, in every lane (DPP row broadcast).
template <int I0, int N, int... Is>
__device__ __forceinline__ void row_words(uint32_t x, uint32_t (&k)[N],
                                          std::integer_sequence<int, Is...>) {
    ((k[Is] = uint32_t(__builtin_amdgcn_mov_dpp(int(x), 0x150 + I0 + Is, 0xf, 0xf, false))), ...);
}

// Middle rounds at positions Q0 .. Q0 + R - 1 of the 12-round sequence below,
// NB blocks.  kq[X] holds, in every row of 16 lanes, the 16 round-key words of
// positions 4X + 1 .. 4X + 4 (lane i: word i % 4 of position 4X + 1 + i / 4);
// a row broadcast (DPP) gives each key word to all lanes as a VGPR, so the
// chunk's rounds hold no round key in SGPRs.
template <bool kInv, int NB, int Q0, int R>
__device__ __forceinline__ void mid_round_chunk(const uint32_t *lds, const Bases &b,
                                                const uint32_t (&kq)[3], uint32_t (&s)[NB][4]) {
    constexpr int kX = (Q0 - 1) / 4;
    constexpr int kI0 = 4 * (Q0 - 1 - 4 * kX);
    static_assert(kI0 + 4 * R <= 16, "a chunk stays within one key register");
    uint32_t k[4 * R];
    row_words<kI0>(kq[kX], k, std::make_integer_sequence<int, 4 * R>{});
#pragma unroll
    for (int t = 0; t < R; ++t) {
#pragma unroll
        for (int j = 0; j < NB; ++j) mid_round<kInv>(lds, b, s[j], &k[4 * t]);
    }
}

// T_t[x] from the table image in device memory (te = its forward tables),
// for an index that is the same in every lane: a scalar load through the
// scalar cache instead of an LDS read.
__device__ __forceinline__ uint32_t table_s(const uint32_t *te, int t, uint32_t x) {
    return as_const(te)[__builtin_amdgcn_readfirstlane(uint32_t(t) * 256u + x)];
}

// Rounds 1 and 2 of a CTR step whose 64 * NB counters start at ctr_first, a
// multiple of 64 * NB (block j of this lane has counter ctr_first + 64 j +
// lane), so they differ only in their low byte.  Round 1 (Eq. (1)): output
// words 1..3 and three terms of word 0 are the same for the whole step; in
// round 2 each output word has one term on word 0 (per block) and three on
// words 1..3 (per step), read once per step through the scalar cache.
template <int NB>
__device__ __forceinline__ void ctr_rounds_1_2(const uint32_t *lds, const uint32_t *te,
                                               const Bases &b, uint32_t kreg,
                                               const CtrConsts &cc, uint32_t ctr_first,
                                               uint32_t lane, uint32_t (&s)[NB][4]) {
    const uint32_t w3u = bswap32(ctr_first) ^ cc.kvar;
    const uint32_t u1 = cc.p[1] ^ table_s(te, 2, (w3u >> 16) & 0xFFu);
    const uint32_t u2 = cc.p[2] ^ table_s(te, 1, (w3u >> 8) & 0xFFu);
    const uint32_t u3 = cc.p[3] ^ table_s(te, 0, w3u & 0xFFu);
    uint32_t k2[4];
    round_key(kreg, 2, k2);
    const uint32_t c0 = xor3(xor3(table_s(te, 1, (u1 >> 8) & 0xFFu),
                                  table_s(te, 2, (u2 >> 16) & 0xFFu), table_s(te, 3, u3 >> 24)),
                             k2[0], 0u);
    const uint32_t c1 = xor3(xor3(table_s(te, 0, u1 & 0xFFu), table_s(te, 1, (u2 >> 8) & 0xFFu),
                                  table_s(te, 2, (u3 >> 16) & 0xFFu)),
                             k2[1], 0u);
    const uint32_t c2 = xor3(xor3(table_s(te, 0, u2 & 0xFFu), table_s(te, 1, (u3 >> 8) & 0xFFu),
                                  table_s(te, 3, u1 >> 24)),
                             k2[2], 0u);
    const uint32_t c3 = xor3(xor3(table_s(te, 0, u3 & 0xFFu), table_s(te, 2, (u1 >> 16) & 0xFFu),
                                  table_s(te, 3, u2 >> 24)),
                             k2[3], 0u);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const uint32_t w3 = bswap32(ctr_first + uint32_t(j) * 64u + lane) ^ cc.kvar;
        const uint32_t v0 = cc.p[0] ^ tlook<3>(lds, w3, b.t[3]);
        s[j][0] = tlook<0>(lds, v0, b.t[0]) ^ c0;
        s[j][1] = tlook<3>(lds, v0, b.t[3]) ^ c1;
        s[j][2] = tlook<2>(lds, v0, b.t[2]) ^ c2;
        s[j][3] = tlook<1>(lds, v0, b.t[1]) ^ c3;
    }
}

// The rounds of one step: NB blocks per lane, block j of this lane at tile
// offset step_off + 64 j + lane (base is the same offset from the message's
// block 0), then the mode's output XOR and the store.
template <bool kInv, int NB, int kPolicy>
__device__ __forceinline__ void crypt_step(const uint32_t *lds, const uint32_t *te, const Bases &b,
                                           uint32_t kreg,
                                           const uint32_t (&kq)[3], uint32_t nr, bool ctr,
                                           const CtrConsts &cc,
                                           const DevMsg &m, uint32_t cbc_mask, uint64_t base,
                                           uint32_t step_off, uint32_t lane, const uint4 (&d)[NB],
                                           const uint4 (&prev)[NB], rsrc_t rout) {
    uint32_t s[NB][4];
    uint32_t rk[4];
    // The rounds up to the last: the standard order, or for whole CTR steps
    // rounds 1 and 2 with their per-step lookups shared.
    auto standard_rounds = [&]() {
        round_key(kreg, 0, rk);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const uint64_t idx = base + uint64_t(j) * 64u + lane;
            if (ctr) {
                counter_round1(lds, b, cc, m.ctr0 + uint32_t(idx), s[j]);
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
            for (int j = 0; j < NB; ++j) mid_round<kInv>(lds, b, s[j], rk);
        }
        if constexpr (NB > 1) {
            // Rounds 2 .. nr - 1 as one straight sequence of 12 rounds that
            // AES-192 enters at its third round and AES-128 at its fifth (round
            // q + nr - 13 at position q), in chunks of two or four rounds whose
            // round keys come from the per-tile key registers by row broadcast.
            // Unlike a rolled loop, or round keys read into SGPRs round by round,
            // this lets the compiler overlap more of the rounds' table reads.
            switch (nr) {
                case 14:
                    mid_round_chunk<kInv, NB, 1, 2>(lds, b, kq, s);
                    [[fallthrough]];
                case 12:
                    mid_round_chunk<kInv, NB, 3, 2>(lds, b, kq, s);
                    [[fallthrough]];
                default:
                    mid_round_chunk<kInv, NB, 5, 4>(lds, b, kq, s);
                    mid_round_chunk<kInv, NB, 9, 4>(lds, b, kq, s);
            }
        } else {
#pragma unroll 1
            for (uint32_t r = 2; r < nr; ++r) {
                round_key(kreg, r, rk);
#pragma unroll
                for (int j = 0; j < NB; ++j) mid_round<kInv>(lds, b, s[j], rk);
            }
        }
    };
    if constexpr (!kInv && NB > 1) {
        if (ctr) {
            // A whole CTR step starts at a counter that is a multiple of
            // 64 * NB (the tile's blocks before the first such counter run
            // in 64-block groups), so rounds 1 and 2 take 5 table reads per
            // block and 15 scalar loads per step, and the sequence enters at
            // round 3.
            ctr_rounds_1_2<NB>(lds, te, b, kreg, cc, m.ctr0 + uint32_t(base), lane, s);
            switch (nr) {
                case 14:
                    mid_round_chunk<false, NB, 2, 2>(lds, b, kq, s);
                    [[fallthrough]];
                case 12:
                    mid_round_chunk<false, NB, 4, 1>(lds, b, kq, s);
                    mid_round_chunk<false, NB, 5, 1>(lds, b, kq, s);
                    [[fallthrough]];
                default:
                    mid_round_chunk<false, NB, 6, 3>(lds, b, kq, s);
                    mid_round_chunk<false, NB, 9, 4>(lds, b, kq, s);
            }
        } else {
            standard_rounds();
        }
    } else {
        standard_rounds();
    }
    round_key(kreg, nr, rk);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if constexpr (kInv)
            last_round_inv(lds, b, s[j], rk);
        else
            last_round_fwd(lds, b, s[j], rk);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        uint4 o = make_uint4(s[j][0], s[j][1], s[j][2], s[j][3]);
        if (ctr) {
            o.x ^= d[j].x;
            o.y ^= d[j].y;
            o.z ^= d[j].z;
            o.w ^= d[j].w;
        }
        if constexpr (kInv) {
            // CBC (Eq. (2)): the ciphertext block before, the IV for block 0.
            // Whole steps find the IV in prev already (run_tile puts it in
            // before the step loop): choosing it here would keep four more
            // SGPRs live through the rounds, and with the SGPRs at their
            // limit the compiler keeps fewer table reads in flight.
            if constexpr (NB == 1) {
                const bool b0 = base + uint64_t(j) * 64u + lane == 0;
                o.x ^= (b0 ? m.nonce[0] : prev[j].x) & cbc_mask;
                o.y ^= (b0 ? m.nonce[1] : prev[j].y) & cbc_mask;
                o.z ^= (b0 ? m.nonce[2] : prev[j].z) & cbc_mask;
                o.w ^= (b0 ? m.ctr0 : prev[j].w) & cbc_mask;
            } else {
                o.x ^= prev[j].x & cbc_mask;
                o.y ^= prev[j].y & cbc_mask;
                o.z ^= prev[j].z & cbc_mask;
                o.w ^= prev[j].w & cbc_mask;
            }
        }
        tile_store16<kPolicy>(rout, (step_off + uint32_t(j) * 64u + lane) * 16u, o);
    }
}

// One tile: nr rounds on BPL blocks per lane per step.  The round loop is not
// unrolled and takes nr at run time: one short loop body serves all key
// sizes, so the code a workgroup runs fits the instruction cache even when
// each CU executes it only once (small batches).  Whole steps of 64 * BPL
// blocks run with the next step's blocks loaded ahead; the blocks after the
// last whole step run 64 at a time, one per lane, so a short tile or a
// tile's ragged end costs rounds only for the waves' 64-block groups that
// hold blocks.
// A wave's last expanded key schedule (lane i holds word i), with the key
// slot and round count it was expanded for.
struct KeyCache {
    uint32_t slot = 0xFFFFFFFFu;
    uint32_t nr = 0;
    uint32_t kreg = 0;
};

template <bool kInv, int BPL, int kPolicy = 0>
__device__ __forceinline__ void run_tile(const uint32_t *lds, const Bases &b, const BatchParams &p,
                                         const DevMsg &m, const Tile &tile,
                                         KeyCache *kc = nullptr) {
    const uint32_t nr = m.nr;
    uint32_t kreg;
    if (kc != nullptr && kc->slot == m.key_slot && kc->nr == nr) {
        // The wave's previous tile had the same key (consecutive tiles of one
        // message, in the queue's order): no expansion.
        kreg = kc->kreg;
    } else if (p.sched) {
        // Resident schedule: lane i loads word i (encryption words first,
        // then the equivalent-inverse-cipher words).
        const uint32_t lane = threadIdx.x & 63u;
        const uint32_t *w = p.sched + uint64_t(m.key_slot) * kSchedWords + (kInv ? 64u : 0u);
        kreg = lane < 4u * (nr + 1) ? w[lane] : 0u;
    } else {
        const uint32_t *key = reinterpret_cast<const uint32_t *>(p.keys + 32ull * m.key_slot);
        kreg = schedule_of<kInv>(lds, b, key, nr);
        if (kc != nullptr) *kc = KeyCache{m.key_slot, nr, kreg};
    }

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
        cc.kvar = k0[3];
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
    // Round keys of the whole steps' middle-round sequence, 16 words per
    // register and row (lane permutes, once per tile): position q runs round
    // q + nr - 13, whose word c is lane 4 (q + nr - 13) + c of the schedule.
    const uint32_t *te = p.tables + kTe;   // forward tables in device memory
    uint32_t kq[3];
#pragma unroll
    for (int x = 0; x < 3; ++x)
        kq[x] = uint32_t(__builtin_amdgcn_ds_bpermute(
            int((4u * (4u * x + 1u) + (lane & 15u) + 4u * (nr - 13u)) * 4u), int(kreg)));
    const uint4 *in = reinterpret_cast<const uint4 *>(p.in + m.in_off);
    uint4 *out = reinterpret_cast<uint4 *>(p.out + m.out_off);
    const uint64_t first = tile.first_block;
    const uint64_t end = first + tile.n_blocks;
    constexpr uint32_t kStep = 64u * BPL;
    const uint64_t lim = end < m.n_full ? end : m.n_full;  // whole blocks of this tile
    // Sizes of buffer resources are read back as wave-uniform values, so that
    // the resources stay in SGPRs.
    const uint32_t n_blk = uniform(lim > first ? uint32_t(lim - first) : 0u);
    // Tile offsets [h0, h1) run in whole steps (all of them at one block per
    // lane), the rest 64 blocks at a time.  A CTR tile's whole steps start at
    // its first block whose counter is a multiple of 64 * BPL.
    uint32_t h0 = 0;
    if (BPL > 1 && ctr) {
        const uint32_t c_first = m.ctr0 + uint32_t(first);
        const uint32_t head = (kStep - c_first % kStep) % kStep;
        h0 = uniform(head < n_blk ? head : n_blk);
    }
    const uint32_t h1 = BPL > 1 ? h0 + (n_blk - h0) / kStep * kStep : n_blk;
    // Buffer resources over the tile's whole blocks: loads past them read
    // zero and stores past them are dropped, so no lane branches and the
    // compiler can wait for exactly the older loads (the next step's blocks
    // are loaded while the current step is computed).  The whole-step loop
    // loads through resources that end at its last step, so its look-ahead
    // past that step reads nothing.
    const rsrc_t rin = buffer_rsrc(in + first, uniform(16u * h1));
    const rsrc_t rout = buffer_rsrc(out + first, 16u * n_blk);
    // CBC decryption (Eq. (2)): every block is XORed with the ciphertext
    // block before it (the IV for block 0), read through a resource that
    // starts one block before the tile.  ECB-decrypt tiles issue the same
    // loads on an empty range, so every tile has the same memory operations.
    const bool cbc = kInv && m.mode == AESGPU_MODE_CBC;
    const uint64_t pbase = first > 0 ? first - 1 : 0;
    const uint32_t pshift = first > 0 ? 0u : 1u;  // block 0 has no predecessor
    const rsrc_t rprev =
        buffer_rsrc(in + pbase, uniform(cbc && h1 ? 16u * (h1 + 1u - pshift) : 0u));
    const uint32_t cbc_mask = cbc ? ~0u : 0u;
    // The blocks outside the whole steps (64 at a time, one per lane) and a
    // CTR message's partial last block run first: nothing they need stays
    // live through the whole steps' rounds, which keeps the SGPRs in use there
    // few enough for the compiler to keep many table reads in flight.
    if constexpr (BPL > 1) {
        if (h0 > 0 || h1 < n_blk) {
            const rsrc_t rin_all = buffer_rsrc(in + first, uniform(16u * n_blk));
            const rsrc_t rprev_all =
                buffer_rsrc(in + pbase, uniform(cbc ? 16u * (n_blk + 1u - pshift) : 0u));
            // Groups start at 0 while below h0 (their stores end at h0), then
            // at h1.
            uint32_t g = h0 > 0 ? 0u : h1;
            uint32_t stop = h0 > 0 ? h0 : n_blk;
            while (g < stop) {
                asm volatile("" : "+v"(kreg));
                uint4 d[1], prev[1];
                d[0] = tile_load16<kPolicy>(rin_all, (g + lane) * 16u);
                prev[0] = make_uint4(0, 0, 0, 0);
                if constexpr (kInv)
                    prev[0] = tile_load16<kPolicy>(rprev_all, (g + lane - pshift) * 16u);
                const rsrc_t rout_g = buffer_rsrc(out + first, uniform(16u * stop));
                crypt_step<kInv, 1, kPolicy>(lds, te, b, kreg, kq, nr, ctr, cc, m, cbc_mask,
                                             first + g, g, lane, d, prev, rout_g);
                g += 64u;
                if (g >= stop && stop != n_blk) {
                    g = h1;
                    stop = n_blk;
                }
            }
        }
    }
    if constexpr (!kInv) {
        // Partial last block of a CTR message (it lies in the message's last
        // tile): every lane computes its keystream, lane q < tail writes byte q.
        if (ctr && m.tail && end > m.n_full) {
            uint32_t s[4];
            uint32_t rk[4];
            counter_round1(lds, b, cc, m.ctr0 + uint32_t(m.n_full), s);
#pragma unroll 1
            for (uint32_t r = 2; r < nr; ++r) {
                round_key(kreg, r, rk);
                mid_round<false>(lds, b, s, rk);
            }
            round_key(kreg, nr, rk);
            last_round_fwd(lds, b, s, rk);
            if (lane < m.tail) {
                const uint8_t *src = reinterpret_cast<const uint8_t *>(in + m.n_full);
                uint8_t *dst = reinterpret_cast<uint8_t *>(out + m.n_full);
                const uint32_t w = lane < 4 ? s[0] : lane < 8 ? s[1] : lane < 12 ? s[2] : s[3];
                dst[lane] = src[lane] ^ uint8_t(w >> (8 * (lane & 3u)));
            }
        }
    }
    uint4 next[BPL], next_prev[BPL];
#pragma unroll
    for (int j = 0; j < BPL; ++j)
        next[j] = tile_load16<kPolicy>(rin, (h0 + uint32_t(j) * 64u + lane) * 16u);
    if constexpr (kInv) {
#pragma unroll
        for (int j = 0; j < BPL; ++j)
            next_prev[j] = tile_load16<kPolicy>(rprev, (h0 + uint32_t(j) * 64u + lane - pshift) * 16u);
        // Message block 0 can only be the first whole step's slot 0 of lane
        // 0 (its predecessor load read nothing): its predecessor is the IV.
        if (first + h0 == 0 && lane == 0)
            next_prev[0] = make_uint4(m.nonce[0], m.nonce[1], m.nonce[2], m.ctr0);
    }
    {
        // In the loop a step's loads are followed by the previous step's
        // stores.  These stores have an empty range and write nothing; they
        // give the loop entry the same order, so the wait at the top of the
        // loop covers the loads only.
        const rsrc_t none = buffer_rsrc(out, 0);
#pragma unroll
        for (int j = 0; j < BPL; ++j)
            tile_store16<kPolicy>(none, (uint32_t(j) * 64u + lane) * 16u, make_uint4(0, 0, 0, 0));
    }
    for (uint32_t step_off = h0; step_off < h1; step_off += kStep) {
        // Keep the round-key reads inside the loop: hoisting all of them would
        // need 4 * (nr + 1) SGPRs at once.
        asm volatile("" : "+v"(kreg));
        uint4 d[BPL], prev[BPL];
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            d[j] = next[j];
            next[j] = tile_load16<kPolicy>(rin, (step_off + kStep + uint32_t(j) * 64u + lane) * 16u);
        }
        if constexpr (kInv) {
#pragma unroll
            for (int j = 0; j < BPL; ++j) {
                prev[j] = next_prev[j];
                next_prev[j] = tile_load16<kPolicy>(
                    rprev, (step_off + kStep + uint32_t(j) * 64u + lane - pshift) * 16u);
            }
        }
        crypt_step<kInv, BPL, kPolicy>(lds, te, b, kreg, kq, nr, ctr, cc, m, cbc_mask, first + step_off,
                                       step_off, lane, d, prev, rout);
    }
}

// S-box applied to each byte of w, per lane, from the lane's own copy of T0
// (byte 1 of T0[x] is S(x)).
__device__ __forceinline__ uint32_t sub_word_lane(const uint32_t *lds, const Bases &b,
                                                  uint32_t w) {
    return ((tlook<0>(lds, w, b.t[0]) >> 8) & 0xFFu) | (tlook<1>(lds, w, b.t[0]) & 0xFF00u) |
           ((tlook<2>(lds, w, b.t[0]) << 8) & 0xFF0000u) |
           ((tlook<3>(lds, w, b.t[0]) << 16) & 0xFF000000u);
}

// Lane q of each group of four lanes receives the value of lane (q + K) mod 4
// of its group (a DPP quad permutation).
template <int K>
__device__ __forceinline__ uint32_t quad_rot(uint32_t v) {
    constexpr int kSel = ((0 + K) & 3) | (((1 + K) & 3) << 2) | (((2 + K) & 3) << 4) |
                         (((3 + K) & 3) << 6);
    return __builtin_amdgcn_update_dpp(0u, v, kSel, 0xF, 0xF, true);
}

// One round of Eq. (1) on a block held by four lanes, lane q holding state
// word q: output word q reads byte k of word q + k (mod 4), which the quad
// permutations bring to lane q.  The last round takes the S-box bytes from
// the T tables as last_round_fwd does.
template <bool kLast>
__device__ __forceinline__ uint32_t quad_round(const uint32_t *lds, const Bases &b, uint32_t s,
                                               uint32_t k) {
    const uint32_t s1 = quad_rot<1>(s), s2 = quad_rot<2>(s), s3 = quad_rot<3>(s);
    if constexpr (kLast)
        return merge4_xor(tlook<0>(lds, s, b.t[2]), tlook<1>(lds, s1, b.t[3]),
                          tlook<2>(lds, s2, b.t[0]), tlook<3>(lds, s3, b.t[1]), k);
    return xor3(xor3(tlook<0>(lds, s, b.t[0]), tlook<1>(lds, s1, b.t[1]),
                     tlook<2>(lds, s2, b.t[2])),
                tlook<3>(lds, s3, b.t[3]), k);
}

// FIPS-197 KeyExpansion of the quad's key; lane q keeps column q of every
// round key (rk[r] = word 4r + q).  Only the last nk words stay live.
template <int NR>
__device__ __forceinline__ void expand_key_quad(const uint32_t *lds, const Bases &b,
                                                const uint32_t (&key)[8], uint32_t q,
                                                uint32_t (&rk)[NR + 1]) {
    constexpr int nk = NR - 6;
    uint32_t win[8];
#pragma unroll
    for (int r = 0; r <= NR; ++r) rk[r] = 0;
#pragma unroll
    for (int i = 0; i < nk; ++i) {
        win[i] = key[i];
        rk[i / 4] = q == uint32_t(i & 3) ? win[i] : rk[i / 4];
    }
    uint32_t rcon = 1;
#pragma unroll
    for (int i = nk; i < 4 * (NR + 1); ++i) {
        uint32_t t = win[(i - 1) % nk];
        if (i % nk == 0) {
            t = sub_word_lane(lds, b, (t >> 8) | (t << 24)) ^ rcon;
            rcon = ((rcon << 1) ^ ((rcon >> 7) * 0x1Bu)) & 0xFFu;
        } else if (nk == 8 && i % nk == 4) {
            t = sub_word_lane(lds, b, t);
        }
        win[i % nk] ^= t;
        rk[i / 4] = q == uint32_t(i & 3) ? win[i % nk] : rk[i / 4];
    }
}

// CBC encryption (C_i = E_K(P_i ^ C_{i-1}), C_{-1} = IV, the inverse of Eq.
// (2)) of a group of up to 16 messages of one key size, four lanes per
// message (lane q of a quad holds column q of the state and of every round
// key).  Blocks of a message are sequential; quads whose message has ended
// compute on and store nothing new (the group is sorted longest first).
// Iteration i stores the previous block and loads the next one before the
// rounds, so the only memory wait (for block i, at the loop top) is on a load
// issued a whole block earlier.
template <int NR>
__device__ void cbc_encrypt_group(const uint32_t *lds, const Bases &b, const BatchParams &p,
                                  const Tile &tile, uint64_t n_max) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t q = lane & 3u;
    const bool active = (lane >> 2) < tile.n_blocks;
    DevMsg m{};
    if (active) m = p.msgs[p.cbc_list[tile.msg + (lane >> 2)]];
    uint32_t rk[NR + 1];
    if (p.sched) {
        const uint32_t *w = p.sched + uint64_t(m.key_slot) * kSchedWords;
#pragma unroll
        for (int r = 0; r <= NR; ++r) rk[r] = w[4 * r + q];
    } else {
        const uint32_t *kp = reinterpret_cast<const uint32_t *>(p.keys + 32ull * m.key_slot);
        uint32_t key[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) key[i] = i < NR - 6 ? kp[i] : 0u;
        expand_key_quad<NR>(lds, b, key, q, rk);
    }
    const uint64_t n = active ? m.n_full : 0;
    const uint64_t last = n ? n - 1 : 0;
    // Every load and store is issued in every iteration (no branch), so the
    // compiler can count them: a quad without a message reads and writes the
    // dummy block; a quad whose message has ended rewrites its last block
    // with the same value.
    const uint32_t *dummy = reinterpret_cast<uint32_t *>(p.cbc_dummy);
    const uint32_t *in = n ? reinterpret_cast<const uint32_t *>(p.in + m.in_off) : dummy;
    uint32_t *out = n ? reinterpret_cast<uint32_t *>(p.out + m.out_off)
                      : reinterpret_cast<uint32_t *>(p.cbc_dummy);
    uint32_t c = q == 0 ? m.nonce[0] : q == 1 ? m.nonce[1] : q == 2 ? m.nonce[2] : m.ctr0;
    uint32_t pt = in[q];
    for (uint64_t i = 0; i < n_max; ++i) {
        uint32_t s = pt ^ c ^ rk[0];
        uint32_t *dst = i == 0 ? reinterpret_cast<uint32_t *>(p.cbc_dummy) + q
                               : out + 4 * (i - 1 < last ? i - 1 : last) + q;
        *dst = c;
        pt = in[4 * (i + 1 <= last ? i + 1 : last) + q];
        // Compiler barrier: keeps the load of the next block issued here,
        // before the rounds, instead of sunk to the next iteration.
        asm volatile("" ::: "memory");
#pragma unroll
        for (int r = 1; r < NR; ++r) s = quad_round<false>(lds, b, s, rk[r]);
        s = quad_round<true>(lds, b, s, rk[NR]);
        // A select, not a branch: c stays live across the rounds, so the
        // register the store above reads is not reused before it is done.
        c = i < n ? s : c;
    }
    if (n) out[4 * last + q] = c;
}

// The CBC-encryption launch: forward tables in LDS, then each wave takes
// every (waves in the grid)-th group from its start (below).  Every wave
// reaches the end of the list.  WG threads per workgroup, one workgroup per
// CU: few waves per CU when there are few groups (each lane's chain of
// blocks is latency-bound), 16 when there are many.
template <int WG>
__global__ __launch_bounds__(WG) void cbc_encrypt_kernel(BatchParams p, const Tile *groups,
                                                         uint32_t n_groups) {
    __shared__ uint32_t lds[kFwdWords];
    stage_tables<false, WG>(lds, p.tables);
    const Bases b = lane_bases();
    // Groups are sorted longest first.  Wave w of workgroup b starts on group
    // w * gridDim.x + b, so the longest groups land on different CUs, each
    // beside shorter ones that finish early: a group's time is its sequential
    // chain, and a chain waits less for the LDS on a CU with fewer waves.
    const uint32_t waves = gridDim.x * (blockDim.x / 64u);
    for (uint32_t g = (threadIdx.x >> 6) * gridDim.x + blockIdx.x; g < n_groups; g += waves) {
        const Tile t = load_uniform(groups + __builtin_amdgcn_readfirstlane(g));
        // The first message is the group's longest; all share one key size.
        const DevMsg m0 = load_uniform(p.msgs + as_const(p.cbc_list)[t.msg]);
        if (m0.nr == 10)
            cbc_encrypt_group<10>(lds, b, p, t, m0.n_full);
        else if (m0.nr == 12)
            cbc_encrypt_group<12>(lds, b, p, t, m0.n_full);
        else
            cbc_encrypt_group<14>(lds, b, p, t, m0.n_full);
    }
}

// Runs tiles of one table set's queue until it is empty.  A wave first runs
// its static tile (`first`, or kNone) and then pulls tiles n_static,
// n_static + 1, ... from the queue's atomic counter, so a launch does no
// atomic at all when every tile has a wave of its own.
constexpr uint32_t kNone = 0xFFFFFFFFu;

// The batch kernel's parameters in its kernel-argument segment (the kernel's
// only argument, at offset 0), through a pointer the compiler cannot assume
// constant from one call to the next, so that each call loads afresh.
__device__ __forceinline__ const BatchParams &kernel_params() {
    const BatchParams __attribute__((address_space(4))) *k =
        (const BatchParams __attribute__((address_space(4))) *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(k));
    return *(const BatchParams *)k;
}

template <bool kInv, int BPL>
__device__ __forceinline__ void drain_queue(const uint32_t *lds, const Bases &b, uint32_t first) {
    constexpr int set = kInv ? 1 : 0;
    uint32_t t = first;
    uint32_t run_end = 0;  // end of the run of tiles taken by the last pull
    KeyCache kc;
    for (;;) {
        // The launch's parameters are read again from the kernel-argument
        // segment for every tile (scalar loads that hit the scalar cache)
        // rather than held in SGPRs through the tile: with fewer SGPRs in use
        // the compiler keeps many more table reads in flight in the rounds.
        const BatchParams &p = kernel_params();
        const DevMsg *__restrict__ msgs = p.msgs;
        const Tile *__restrict__ tiles = p.tiles[set];
        t = __builtin_amdgcn_readfirstlane(t);
        if (t == kNone) {
            if (p.n_static[set] >= p.n_tiles[set]) break;  // no dynamic tiles at all
            // One atomic per run of `pull` consecutive tiles (similar in size,
            // the queue being sorted): all waves of the chip pull from one
            // counter, whose atomics would otherwise bound batches of many
            // short tiles.
            uint32_t c = 0;
            if ((threadIdx.x & 63u) == 0) c = atomicAdd(&p.counters[set], p.pull[set]);
            t = p.n_static[set] + __builtin_amdgcn_readfirstlane(c);
            run_end = t + p.pull[set];
        }
        if (t >= p.n_tiles[set]) break;
        // Scalar loads (the index is wave-uniform and nothing writes the
        // descriptors during a launch), so every field is uniform.
        const Tile tile = load_uniform(tiles + t);
        const DevMsg m = load_uniform(msgs + tile.msg);
        run_tile<kInv, BPL>(lds, b, p, m, tile, &kc);
        t = t + 1 < run_end ? t + 1 : kNone;
    }
}

// One launch for both table sets: workgroups below n_wg_forward_first start
// on the forward queue, the others on the inverse queue; wave w of the i-th
// workgroup of a set owns static tile 16 i + w of that set.  A workgroup
// whose queue runs dry waits until all its waves are done with the LDS
// tables, then stages the other set and helps drain the other queue (if
// tiles are left there).
template <int BPL>
__global__ __launch_bounds__(kWG) void batch_kernel(BatchParams p) {
    __shared__ uint32_t lds[kFwdWords + kInvSWords];
    const Bases b = lane_bases();
    const uint32_t first = blockIdx.x < p.n_wg_forward_first ? 0u : 1u;
    const uint32_t wg_in_set = first ? blockIdx.x - p.n_wg_forward_first : blockIdx.x;
    const uint32_t my_static = wg_in_set * (kWG / 64) + (threadIdx.x >> 6);
    for (uint32_t pass = 0; pass < 2; ++pass) {
        const uint32_t set = pass ^ first;
        // Stage the set only if this workgroup has work in it: a static tile
        // (first pass) or dynamic tiles still queued.  One thread decides and
        // publishes the decision in this workgroup's flag word (the LDS is
        // full), so that every wave takes the same branch.
        uint32_t *flag = p.counters + 2 + blockIdx.x;
        __syncthreads();  // all waves are past the previous queue
        if (threadIdx.x == 0) {
            const uint32_t pulled =
                __hip_atomic_load(&p.counters[set], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool has_static = pass == 0 && wg_in_set * (kWG / 64) < p.n_tiles[set];
            const bool has_dynamic = p.n_static[set] < p.n_tiles[set] &&
                                     pulled < p.n_tiles[set] - p.n_static[set];
            __hip_atomic_store(flag, (has_static || has_dynamic) ? 1u : 0u, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (!__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) continue;
        const uint32_t start = (pass == 0 && my_static < p.n_tiles[set]) ? my_static : kNone;
        // The staging's indices and addresses are recomputed here rather than
        // kept in registers through the whole launch.
        const uint32_t *tables = p.tables;
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+s"(tables), "+v"(tid));
        if (set == 0) {
            stage_tables_tid<false>(lds, tables, tid);
            drain_queue<false, BPL>(lds, b, start);
        } else {
            stage_tables_tid<true>(lds, tables, tid);
            drain_queue<true, BPL>(lds, b, start);
        }
    }
    // The last workgroup to finish zeroes the two queue counters (and the
    // exit count), so the next launch on these counters needs no reset
    // kernel before it: every workgroup counts itself out after its last
    // pull, so no pull of this launch can follow the reset.
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t *exits = p.counters + kExitWord;
        const uint32_t before = __hip_atomic_fetch_add(exits, 1u, __ATOMIC_ACQ_REL,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        if (before == gridDim.x - 1) {
            __hip_atomic_store(&p.counters[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&p.counters[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(exits, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---- resident serving kernel ---------------------------------------------------
//
// The kernel stays on the GPU while requests keep coming: the host writes
// tile records into two rings in pinned host memory (ring 0 for the forward
// tables, ring 1 for the inverse tables) and publishes each ring's tail;
// workgroups below n_wg_forward serve ring 0, the others ring 1, each with
// its table set staged once.  Wave 0 of the first workgroup of each set reads
// the host's tail and stop words over the link and copies its ring's tail into
// every workgroup's copy block (which holds both rings' tails, so a workgroup
// that serves the other ring after a relaunch never reads a tail of the
// wrong ring); the other waves watch their workgroup's copy.
// A wave takes tiles by tickets: one fetch-and-add on its set's claim counter
// (a compare-and-swap there serialises thousands of waves), taken only while
// the copy shows tiles that no ticket covers yet.  A ticket may run ahead of
// the published tail: its wave then waits for the host to publish that tile,
// so at most one ticket per wave is ahead.  The wave that counts a request's
// last tile (each request slot has a tile counter that only grows; a record
// carries the count that completes its request) appends the slot to a
// completion ring in host memory, each entry tagged with its position so
// that the host reads the ring in order.
// Tiles load and store with the agent-coherent cache policy, so a tile sees
// its input and publishes its output device-wide with no per-tile fence (an
// L2 invalidation or write-back at this scope, which would serialise).
// Tickets ahead of the tail are bounded: a wave takes one only while the
// claim counter is less than the tail plus twice its set's workgroups, so a
// new tail at low load does not send every idle wave of the set to wait on a
// tile of its own.
// Every wave ends, and only on its set's stop word: the poller ends after the
// host's stop word or idle_polls polls without a new tail and then posts the
// launch epoch in every stop word of its set; a worker ends once that word
// holds the epoch (after serving a ticket that is published by then).  A
// worker never leaves on a timer of its own: a ticket it gave up would be
// below a later tail and never served, and a set whose workers had left
// would leave its poller publishing tiles that nobody takes.  (Workgroups
// are dispatched in order of their index, so each set's poller, in the
// set's first workgroup, is resident before any of its workers.)  The last
// wave to end points each claim counter back at the first tile that no wave
// served (tickets that ran ahead and were never published), so the next
// launch starts there.

constexpr uint64_t kNoTile = ~0ull;

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return (uint64_t(hi) << 32) | lo;
}

// A tile record from host memory: lanes 0..15 read one word each, bypassing
// the caches (ring entries are rewritten by the host), then every field is
// made wave-uniform.
__device__ __forceinline__ ResTile load_record(const ResTile *r) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t *w = reinterpret_cast<uint32_t *>(const_cast<ResTile *>(r));
    uint32_t v = 0;
    if (lane < 16) v = __hip_atomic_load(w + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    ResTile t;
    uint32_t *d = reinterpret_cast<uint32_t *>(&t);
#pragma unroll
    for (int i = 0; i < 16; ++i) d[i] = __builtin_amdgcn_readlane(v, i);
    return t;
}

// The set's poller: its ring's host tail, copied to every workgroup, and the
// host's stop word, passed on as this launch's epoch to its set's
// workgroups.
__device__ void poll_host(const ResidentLaunch &p, uint32_t set) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wg0 = set ? p.n_wg_forward : 0u, wg1 = set ? p.n_wg : p.n_wg_forward;
    uint64_t *host = const_cast<uint64_t *>(p.host_ctl);
    uint64_t seen = 0;
    uint32_t idle = 0;
    for (;;) {
        uint64_t h = 0, stop = 0;
        // Relaxed loads that bypass the caches: the tile records are read
        // the same way, so no acquire (an L2 invalidation) is needed here.
        if (lane == 0) {
            h = __hip_atomic_load(host + set, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            stop = __hip_atomic_load(host + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        h = uniform64(h);
        stop = uniform64(stop);
        if (h > seen) {
            for (uint32_t w = lane; w < p.n_wg; w += 64)
                __hip_atomic_store(p.dev + kResCopyWord + 16 * size_t(w) + set, h,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            seen = h;
            idle = 0;
        }
        if (stop || ++idle > p.idle_polls) {
            // Release: a worker that sees the stop word also sees every tail
            // stored before it.
            for (uint32_t w = wg0 + lane; w < wg1; w += 64)
                __hip_atomic_store(p.dev + kResCopyWord + 16 * size_t(w) + 2,
                                   uint64_t(p.epoch), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

// A worker wave of one set: take tickets, run and count tiles until told to
// stop.
template <bool kInv, int BPL>
__device__ void serve_ring(const uint32_t *lds, const Bases &b, const ResidentLaunch &p) {
    constexpr uint32_t set = kInv ? 1u : 0u;
    const uint32_t lane = threadIdx.x & 63u;
    uint64_t *claimed = p.dev + 16 * set;
    uint64_t *copy = p.dev + kResCopyWord + 16 * size_t(blockIdx.x);
    BatchParams bp{};
    bp.sched = p.sched;
    bp.tables = p.tables;
    uint64_t known = 0;         // tickets reached this tail when last taken
    uint64_t ticket = kNoTile;  // this wave's tile, perhaps not yet published
    const uint64_t ahead = 2ull * (kInv ? p.n_wg - p.n_wg_forward : p.n_wg_forward);
    for (;;) {
        // Relaxed polls: an acquire at this scope invalidates the L2, which
        // thousands of polling waves must not do.
        uint64_t tl = 0, st = 0;
        if (lane == 0) {
            tl = __hip_atomic_load(copy + set, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st = __hip_atomic_load(copy + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        tl = uniform64(tl);
        st = uniform64(st);
        if (st >= p.epoch) {
            // Stopping: the tail stored before the stop word is visible now.
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (lane == 0)
                tl = __hip_atomic_load(copy + set, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tl = uniform64(tl);
            if (ticket == kNoTile || ticket >= tl) break;
        }
        if (ticket == kNoTile && tl > known) {
            uint64_t t = kNoTile;
            if (lane == 0) {
                const uint64_t c = __hip_atomic_load(claimed, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                if (c < tl + ahead)
                    t = __hip_atomic_fetch_add(claimed, 1ull, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
            }
            ticket = uniform64(t);
            // No ticket, or one at or past the tail: every published tile
            // has a ticket.
            if (ticket == kNoTile || ticket >= tl) known = tl;
        }
        if (ticket != kNoTile && ticket < tl) {
            const ResTile r = load_record(p.ring[set] + (ticket & p.ring_mask));
            ticket = kNoTile;
            DevMsg m{};
            m.in_off = r.in;     // absolute addresses: bp.in and bp.out are null
            m.out_off = r.out;
            m.n_full = r.n_blocks;
            m.key_slot = r.key_slot;
            m.nr = r.nr;
            m.mode = AESGPU_MODE_ECB;
            const Tile tile{0u, r.n_blocks, 0ull};
            // Agent-coherent loads and stores: the tile reads its input as the
            // producer left it and its output is visible device-wide once the
            // stores are complete, with no L2 invalidation or write-back (a
            // fence at this scope costs one per tile, and those serialise).
            run_tile<kInv, BPL, kCoherent>(lds, b, bp, m, tile);
            // The tile is counted once its stores are complete.  The slot's
            // counter only grows (modulo 2^32); the record holds the count at
            // which this request is complete, and the wave that reaches it
            // reports the request to the host, which reads no output data.
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (lane == 0) {
                const uint32_t n = __hip_atomic_fetch_add(p.tiles_done + r.req_slot, 1u,
                                                          __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT) + 1u;
                if (n == r.target) {
                    const uint64_t i = __hip_atomic_fetch_add(p.dev + kResDoneWord, 1ull,
                                                              __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(p.done_ring + (i & p.done_mask),
                                       ((i + 1) << 32) | r.req_slot, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
            continue;
        }
        // Nothing to run: wait for a new tail or the stop word (a wave
        // holding a ticket polls more often, its tile comes next).
        if (ticket == kNoTile)
            __builtin_amdgcn_s_sleep(32);
        else
            __builtin_amdgcn_s_sleep(2);
    }
}

template <int BPL>
__global__ __launch_bounds__(kWG) void resident_kernel(ResidentLaunch p) {
    __shared__ uint32_t lds[kFwdWords + kInvSWords];
    const Bases b = lane_bases();
    const bool inv = blockIdx.x >= p.n_wg_forward;   // uniform over the workgroup
    if (inv)
        stage_tables<true>(lds, p.tables);
    else
        stage_tables<false>(lds, p.tables);
    if ((threadIdx.x >> 6) == 0 && (blockIdx.x == 0 || blockIdx.x == p.n_wg_forward))
        poll_host(p, inv ? 1u : 0u);
    else if (inv)
        serve_ring<true, BPL>(lds, b, p);
    else
        serve_ring<false, BPL>(lds, b, p);
    // Count the wave out.  The last one points each claim counter at the
    // first tile no wave served: tickets beyond the last published tail were
    // never served, every ticket below it was.
    if ((threadIdx.x & 63u) == 0) {
        const uint64_t waves = uint64_t(gridDim.x) * (kWG / 64);
        const uint64_t before = __hip_atomic_fetch_add(p.dev + kResExitWord, 1ull,
                                                       __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (before == waves - 1) {
            for (uint32_t set = 0; set < 2; ++set) {
                const uint64_t seen = __hip_atomic_load(p.dev + kResCopyWord + set,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t c = __hip_atomic_load(p.dev + 16 * set, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                if (c > seen)
                    __hip_atomic_store(p.dev + 16 * set, seen, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
            __hip_atomic_store(p.dev + kResExitWord, 0ull, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int BPL>
int enqueue_t(const BatchLaunch &L, hipStream_t s) {
    const uint32_t total = L.n_tiles[0] + L.n_tiles[1];
    if (!total && !L.n_cbc_groups) return AESGPU_OK;
    // About one tile per wave for small batches, one workgroup per CU at most.
    constexpr uint32_t kWaves = kWG / 64;
    uint32_t grid = (total + kWaves - 1) / kWaves;
    if (grid > uint32_t(L.n_cu)) grid = uint32_t(L.n_cu);
    if (grid > 1024) grid = 1024;  // one flag word per workgroup in the counter area
    if (grid < 2 && L.n_tiles[0] && L.n_tiles[1]) grid = 2;
    // Split the workgroups between the queues in proportion to their blocks.
    uint32_t fwd = 0;
    if (!L.n_tiles[1]) {
        fwd = grid;
    } else if (L.n_tiles[0]) {
        const double share = double(L.blocks[0]) / double(L.blocks[0] + L.blocks[1]);
        fwd = uint32_t(share * grid + 0.5);
        fwd = fwd < 1 ? 1 : (fwd > grid - 1 ? grid - 1 : fwd);
    }
    // Dynamic tiles per pull: about four pulls per wave of the grid for each
    // queue, at most 32 tiles.
    uint32_t pull[2] = {1u, 1u};
    const uint32_t n_static[2] = {fwd * kWaves, (grid - fwd) * kWaves};
    for (int q = 0; q < 2 && grid; ++q) {  // grid is 0 when only CBC encryption runs
        const uint32_t dyn = L.n_tiles[q] > n_static[q] ? L.n_tiles[q] - n_static[q] : 0u;
        pull[q] = std::min<uint32_t>(32u, std::max<uint32_t>(1u, dyn / (grid * kWaves * 4u)));
    }
    BatchParams p{L.msgs,     {L.tiles[0], L.tiles[1]}, {L.n_tiles[0], L.n_tiles[1]},
                  L.counters, fwd,  {n_static[0], n_static[1]}, {pull[0], pull[1]},
                  L.keys,     L.sched, L.in, L.out, L.tables, L.cbc_list, L.cbc_dummy};
    // Each launch's own status (the thread's last-error state may hold an
    // earlier, unrelated failure).
    if (L.n_tiles[0] + L.n_tiles[1]) {
        void *args[] = {&p};
        if (hipLaunchKernel(reinterpret_cast<const void *>(&batch_kernel<BPL>), dim3(grid),
                            dim3(kWG), args, 0, s) != hipSuccess)
            return AESGPU_EHIP;
    }
    if (L.n_cbc_groups) {
        const uint32_t n_cu = uint32_t(L.n_cu);
        const Tile *groups = L.cbc_groups;
        uint32_t n_groups = L.n_cbc_groups;
        void *args[] = {&p, &groups, &n_groups};
        hipError_t e;
        if (n_groups <= 4 * n_cu) {
            const uint32_t g = (n_groups + 3) / 4;
            e = hipLaunchKernel(reinterpret_cast<const void *>(&cbc_encrypt_kernel<256>), dim3(g),
                                dim3(256), args, 0, s);
        } else {
            const uint32_t g = std::min<uint32_t>((n_groups + 15) / 16, n_cu);
            e = hipLaunchKernel(reinterpret_cast<const void *>(&cbc_encrypt_kernel<kWG>), dim3(g),
                                dim3(kWG), args, 0, s);
        }
        if (e != hipSuccess) return AESGPU_EHIP;
    }
    return AESGPU_OK;
}

}  // namespace

int enqueue_batch(const BatchLaunch &L, hipStream_t s) {
    return L.bpl == 1 ? enqueue_t<1>(L, s) : L.bpl == 2 ? enqueue_t<2>(L, s) : enqueue_t<4>(L, s);
}

int launch_resident(const ResidentLaunch &L, hipStream_t s) {
    if (L.n_wg < 2 || L.n_wg > 1024 || L.n_wg_forward == 0 || L.n_wg_forward >= L.n_wg ||
        L.epoch == 0 || (L.ring_mask & (L.ring_mask + 1)) != 0 ||
        (L.done_mask & (L.done_mask + 1)) != 0)
        return AESGPU_EINVAL;
    ResidentLaunch p = L;
    void *args[] = {&p};
    const void *fn = L.bpl == 1   ? reinterpret_cast<const void *>(&resident_kernel<1>)
                     : L.bpl == 2 ? reinterpret_cast<const void *>(&resident_kernel<2>)
                                  : reinterpret_cast<const void *>(&resident_kernel<4>);
    return hipLaunchKernel(fn, dim3(L.n_wg), dim3(kWG), args, 0, s) == hipSuccess ? AESGPU_OK
                                                                                 : AESGPU_EHIP;
}

int build_tiles(const aesgpu_msg *msgs, size_t m, uint32_t tile_blocks, std::vector<DevMsg> &dm,
                std::vector<Tile> (&tiles)[2], std::vector<uint32_t> &cbc_list,
                std::vector<Tile> &cbc_groups, BatchTotals &tot) {
    dm.resize(m);
    tiles[0].clear();
    tiles[1].clear();
    cbc_list.clear();
    cbc_groups.clear();
    tot = BatchTotals{};
    std::vector<uint32_t> cbc_enc[3];   // CBC-encrypt messages per key size
    for (size_t i = 0; i < m; ++i) {
        const aesgpu_msg &x = msgs[i];
        if (x.key_bits != 128 && x.key_bits != 192 && x.key_bits != 256) return AESGPU_EKEYLEN;
        if (x.mode != AESGPU_MODE_ECB && x.mode != AESGPU_MODE_CTR && x.mode != AESGPU_MODE_CBC)
            return AESGPU_EINVAL;
        if (x.dir != AESGPU_DIR_ENCRYPT && x.dir != AESGPU_DIR_DECRYPT) return AESGPU_EINVAL;
        if ((x.in_off & 15u) || (x.out_off & 15u)) return AESGPU_EALIGN;
        if (x.mode != AESGPU_MODE_CTR && (x.n_bytes & 15u)) return AESGPU_EINVAL;
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
        d.ctr0 = x.ctr0;   // CBC: IV bytes 12..15 as a little-endian word
        tot.total += x.n_bytes;
        if (x.n_bytes) {
            tot.in_end = std::max(tot.in_end, x.in_off + x.n_bytes);
            tot.out_end = std::max(tot.out_end, x.out_off + x.n_bytes);
            tot.max_slot = std::max(tot.max_slot, x.key_slot);
        }
        if (x.mode == AESGPU_MODE_CBC && x.dir == AESGPU_DIR_ENCRYPT) {
            if (n_blocks) cbc_enc[(x.key_bits - 128) / 64].push_back(uint32_t(i));
            continue;
        }
        const bool inverse = x.mode != AESGPU_MODE_CTR && x.dir == AESGPU_DIR_DECRYPT;
        if (x.mode == AESGPU_MODE_CBC && inverse && x.n_bytes &&
            x.in_off < x.out_off + x.n_bytes && x.out_off < x.in_off + x.n_bytes)
            tot.cbc_dec_self_overlap = true;
        const int set = inverse ? 1 : 0;
        tot.blocks[set] += n_blocks;
        // A CTR message's first tile ends where the counter reaches a multiple
        // of 256 (when the tile size is one), so that every later tile starts
        // there: the kernel runs a tile's whole steps from such a counter on
        // and the blocks before it in 64-block groups.
        uint64_t first_len = tile_blocks;
        if (x.mode == AESGPU_MODE_CTR && tile_blocks % 256u == 0) {
            const uint64_t cut = tile_blocks - (uint64_t(x.ctr0) + tile_blocks) % 256u;
            if (cut > 0) first_len = cut;
        }
        for (uint64_t f = 0; f < n_blocks;) {
            const uint64_t n = std::min<uint64_t>(f ? tile_blocks : first_len, n_blocks - f);
            tiles[set].push_back(Tile{uint32_t(i), uint32_t(n), f});
            f += n;
        }
    }
    for (auto &t : tiles)
        std::stable_sort(t.begin(), t.end(),
                         [](const Tile &a, const Tile &b) { return a.n_blocks > b.n_blocks; });
    // CBC-encrypt groups: per key size, longest first, 16 messages (four
    // lanes each) per group; all groups longest first, since each runs its blocks one
    // after another.
    for (auto &v : cbc_enc) {
        std::stable_sort(v.begin(), v.end(), [&](uint32_t a, uint32_t b) {
            return dm[a].n_full > dm[b].n_full;
        });
        for (size_t g = 0; g < v.size(); g += kCbcGroupMsgs) {
            const size_t n = std::min<size_t>(kCbcGroupMsgs, v.size() - g);
            cbc_groups.push_back(Tile{uint32_t(cbc_list.size()), uint32_t(n), dm[v[g]].n_full});
            cbc_list.insert(cbc_list.end(), v.begin() + long(g), v.begin() + long(g + n));
        }
    }
    std::stable_sort(cbc_groups.begin(), cbc_groups.end(),
                     [](const Tile &a, const Tile &b) { return a.first_block > b.first_block; });
    return AESGPU_OK;
}

}  // namespace aesgpu

using namespace aesgpu;

namespace {
constexpr uint32_t kDefaultBpl = 4;
constexpr uint32_t kDefaultTileBlocks = 8192;
}  // namespace

// Descriptor scratch of aesgpu_batch_run_noalloc(): one copy on each GPU the
// library runs on, held until the process ends.  In host code this name is a
// host-side stand-in, not a device address: host code uses only the address
// hipGetSymbolAddress returns for the current device (scratch_address()).
static __device__ __align__(256) uint8_t scratch[AESGPU_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of this GPU's scratch, looked up once per device with
// that device current (each GPU holds its own copy at its own address).
void *scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

struct aesgpu_batch {
    aesgpu_ctx *ctx = nullptr;
    uint32_t bpl = kDefaultBpl;
    uint32_t tile_blocks = kDefaultTileBlocks;
    bool use_graph = true;
    size_t n_msgs = 0;
    size_t n_tiles[2] = {0, 0};    // forward, inverse
    BatchTotals tot;
    void *d_mem = nullptr;         // messages | forward tiles | inverse tiles | counters
    DevMsg *d_msgs = nullptr;
    Tile *d_tiles[2] = {nullptr, nullptr};
    uint32_t *d_counters = nullptr;
    Tile *d_cbc_groups = nullptr;
    uint32_t *d_cbc_list = nullptr;
    uint4 *d_cbc_dummy = nullptr;
    size_t n_cbc_groups = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *cap_keys = nullptr, *cap_in = nullptr;
    void *cap_out = nullptr;
};

namespace {

// Checks of a run's buffers against a planned batch's totals (every
// message inside d_in / d_out, key slots present, no partial overlap).
int check_run(const BatchTotals &tot, const uint8_t *d_keys, size_t n_key_slots,
              const void *d_in, size_t in_bytes, const void *d_out, size_t out_bytes) {
    if (!d_keys || !d_in || !d_out) return AESGPU_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_keys) | reinterpret_cast<uintptr_t>(d_in) |
         reinterpret_cast<uintptr_t>(d_out)) & 15u)
        return AESGPU_EALIGN;
    if (uint64_t(tot.max_slot) >= n_key_slots) return AESGPU_EINVAL;
    if (tot.in_end > in_bytes || tot.out_end > out_bytes) return AESGPU_EINVAL;
    const uintptr_t i0 = reinterpret_cast<uintptr_t>(d_in), o0 = reinterpret_cast<uintptr_t>(d_out);
    if (i0 != o0 && i0 < o0 + out_bytes && o0 < i0 + in_bytes) return AESGPU_EINVAL;
    if (i0 == o0 && tot.cbc_dec_self_overlap) return AESGPU_EINVAL;
    return AESGPU_OK;
}

// The launch shape a config asks for (NULL: the defaults).
int batch_shape(const aesgpu_batch_config *cfg, uint32_t &bpl, uint32_t &tile_blocks,
                bool &use_graph) {
    bpl = kDefaultBpl;
    tile_blocks = kDefaultTileBlocks;
    use_graph = true;
    if (cfg) {
        if (cfg->blocks_per_lane) bpl = cfg->blocks_per_lane;
        if (cfg->tile_blocks) tile_blocks = cfg->tile_blocks;
        use_graph = !(cfg->flags & AESGPU_BATCH_NO_GRAPH);
    }
    if (bpl != 1 && bpl != 2 && bpl != 4) return AESGPU_EINVAL;
    if (tile_blocks % (64u * bpl) != 0 || tile_blocks > (1u << 24)) return AESGPU_EINVAL;
    return AESGPU_OK;
}

void release_graph(aesgpu_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

int enqueue(aesgpu_batch *b, const uint8_t *keys, const void *in, void *out, hipStream_t s) {
    BatchLaunch L{};
    L.msgs = b->d_msgs;
    L.tiles[0] = b->d_tiles[0];
    L.tiles[1] = b->d_tiles[1];
    L.n_tiles[0] = uint32_t(b->n_tiles[0]);
    L.n_tiles[1] = uint32_t(b->n_tiles[1]);
    L.counters = b->d_counters;
    L.keys = keys;
    L.sched = nullptr;
    L.in = static_cast<const uint8_t *>(in);
    L.out = static_cast<uint8_t *>(out);
    L.tables = b->ctx->d_tables;
    L.cbc_list = b->d_cbc_list;
    L.cbc_groups = b->d_cbc_groups;
    L.cbc_dummy = b->d_cbc_dummy;
    L.n_cbc_groups = uint32_t(b->n_cbc_groups);
    L.n_cu = b->ctx->n_cu;
    L.bpl = b->bpl;
    L.blocks[0] = b->tot.blocks[0];
    L.blocks[1] = b->tot.blocks[1];
    return enqueue_batch(L, s);
}

}  // namespace

extern "C" {

int aesgpu_batch_plan(aesgpu_ctx *ctx, const aesgpu_msg *msgs, size_t m,
                      const aesgpu_batch_config *cfg, aesgpu_batch **out) {
    if (!out) return AESGPU_EINVAL;
    *out = nullptr;
    if (!ctx || (m > 0 && !msgs)) return AESGPU_EINVAL;
    if (m > 0xFFFFFFFFull) return AESGPU_EINVAL;
    uint32_t bpl, tile_blocks;
    bool use_graph;
    const int shape = batch_shape(cfg, bpl, tile_blocks, use_graph);
    if (shape != AESGPU_OK) return shape;

    std::vector<DevMsg> dm;
    std::vector<Tile> tiles[2];
    std::vector<uint32_t> cbc_list;
    std::vector<Tile> cbc_groups;
    BatchTotals tot;
    const int st = build_tiles(msgs, m, tile_blocks, dm, tiles, cbc_list, cbc_groups, tot);
    if (st != AESGPU_OK) return st;
    if (tiles[0].size() > 0xFFFFFFFFull || tiles[1].size() > 0xFFFFFFFFull ||
        cbc_groups.size() > 0xFFFFFFFFull)
        return AESGPU_EINVAL;

    aesgpu_batch *b = new (std::nothrow) aesgpu_batch;
    if (!b) return AESGPU_ENOMEM;
    b->ctx = ctx;
    b->bpl = bpl;
    b->tile_blocks = tile_blocks;
    b->use_graph = use_graph;
    b->n_msgs = m;
    b->n_tiles[0] = tiles[0].size();
    b->n_tiles[1] = tiles[1].size();
    b->n_cbc_groups = cbc_groups.size();
    b->tot = tot;

    DeviceGuard g(ctx->device);
    if (!g.ok()) {
        delete b;
        return AESGPU_EHIP;
    }
    const size_t msg_bytes = m * sizeof(DevMsg);
    const size_t t0 = tiles[0].size() * sizeof(Tile), t1 = tiles[1].size() * sizeof(Tile);
    const size_t cg = cbc_groups.size() * sizeof(Tile);
    const size_t cl = cbc_list.size() * sizeof(uint32_t);
    const size_t dummy = cg ? 16 : 0;
    const size_t bytes = msg_bytes + t0 + t1 + kCounterBytes + cg + dummy + cl;
    if (hipMalloc(&b->d_mem, bytes) != hipSuccess) {
        delete b;
        return AESGPU_ENOMEM;
    }
    char *base = static_cast<char *>(b->d_mem);
    b->d_msgs = reinterpret_cast<DevMsg *>(base);
    b->d_tiles[0] = reinterpret_cast<Tile *>(base + msg_bytes);
    b->d_tiles[1] = reinterpret_cast<Tile *>(base + msg_bytes + t0);
    b->d_counters = reinterpret_cast<uint32_t *>(base + msg_bytes + t0 + t1);
    b->d_cbc_groups = reinterpret_cast<Tile *>(base + msg_bytes + t0 + t1 + kCounterBytes);
    b->d_cbc_dummy = reinterpret_cast<uint4 *>(base + msg_bytes + t0 + t1 + kCounterBytes + cg);
    b->d_cbc_list =
        reinterpret_cast<uint32_t *>(base + msg_bytes + t0 + t1 + kCounterBytes + cg + dummy);
    bool ok = true;
    if (cg)
        ok &= hipMemcpy(b->d_cbc_groups, cbc_groups.data(), cg, hipMemcpyHostToDevice) ==
              hipSuccess;
    if (!cbc_list.empty())
        ok &= hipMemcpy(b->d_cbc_list, cbc_list.data(), cbc_list.size() * sizeof(uint32_t),
                        hipMemcpyHostToDevice) == hipSuccess;
    if (msg_bytes) ok &= hipMemcpy(b->d_msgs, dm.data(), msg_bytes, hipMemcpyHostToDevice) == hipSuccess;
    if (t0) ok &= hipMemcpy(b->d_tiles[0], tiles[0].data(), t0, hipMemcpyHostToDevice) == hipSuccess;
    if (t1) ok &= hipMemcpy(b->d_tiles[1], tiles[1].data(), t1, hipMemcpyHostToDevice) == hipSuccess;
    // The queue counters start at zero once; every launch leaves them zero.
    const std::vector<uint8_t> zeros(kCounterBytes, 0);
    ok &= hipMemcpy(b->d_counters, zeros.data(), kCounterBytes, hipMemcpyHostToDevice) ==
          hipSuccess;
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
    if (b->n_tiles[0] + b->n_tiles[1] + b->n_cbc_groups == 0) return AESGPU_OK;
    const int chk = check_run(b->tot, d_keys, n_key_slots, d_in, in_bytes, d_out, out_bytes);
    if (chk != AESGPU_OK) return chk;
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
    out->total_bytes = b->tot.total;
    out->in_bytes_needed = b->tot.in_end;
    out->out_bytes_needed = b->tot.out_end;
    out->blocks_per_lane = b->bpl;
    out->tile_blocks = b->tile_blocks;
    out->launches = ((b->n_tiles[0] + b->n_tiles[1]) ? 1u : 0u) + (b->n_cbc_groups ? 1u : 0u);
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

int aesgpu_batch_run_noalloc(aesgpu_ctx *ctx, const aesgpu_msg *msgs, size_t m,
                             const aesgpu_batch_config *cfg, const uint8_t *d_keys,
                             size_t n_key_slots, const void *d_in, size_t in_bytes, void *d_out,
                             size_t out_bytes, aesgpu_stream_t stream) {
    if (!ctx || (m > 0 && !msgs)) return AESGPU_EINVAL;
    if (m > 0xFFFFFFFFull) return AESGPU_EINVAL;
    uint32_t bpl, tile_blocks;
    bool use_graph;
    const int shape = batch_shape(cfg, bpl, tile_blocks, use_graph);
    if (shape != AESGPU_OK) return shape;
    // Host-side planning reuses this thread's buffers from call to call.
    thread_local std::vector<DevMsg> dm;
    thread_local std::vector<Tile> tiles[2];
    thread_local std::vector<uint32_t> cbc_list;
    thread_local std::vector<Tile> cbc_groups;
    thread_local std::vector<uint8_t> staging;
    BatchTotals tot;
    const int st = build_tiles(msgs, m, tile_blocks, dm, tiles, cbc_list, cbc_groups, tot);
    if (st != AESGPU_OK) return st;
    if (tiles[0].size() + tiles[1].size() + cbc_groups.size() == 0) return AESGPU_OK;
    const int chk = check_run(tot, d_keys, n_key_slots, d_in, in_bytes, d_out, out_bytes);
    if (chk != AESGPU_OK) return chk;
    // Scratch layout, each part 256-byte aligned: queue counters (zero, as the
    // batch kernel expects before a launch), messages, forward tiles, inverse
    // tiles, CBC-encryption groups, 16 dummy bytes, CBC list.
    const size_t o_msgs = align256(kCounterBytes);
    const size_t o_t0 = o_msgs + align256(m * sizeof(DevMsg));
    const size_t o_t1 = o_t0 + align256(tiles[0].size() * sizeof(Tile));
    const size_t o_cg = o_t1 + align256(tiles[1].size() * sizeof(Tile));
    const size_t o_dummy = o_cg + align256(cbc_groups.size() * sizeof(Tile));
    const size_t o_cl = o_dummy + 256;
    const size_t total = o_cl + cbc_list.size() * sizeof(uint32_t);
    if (total > AESGPU_NOALLOC_SCRATCH_BYTES) return AESGPU_ESCRATCH;
    // The queue counters must start at zero; the padding between parts is
    // never read.
    staging.resize(total);
    uint8_t *h = staging.data();
    std::memset(h, 0, kCounterBytes);
    if (m) std::memcpy(h + o_msgs, dm.data(), m * sizeof(DevMsg));
    if (!tiles[0].empty()) std::memcpy(h + o_t0, tiles[0].data(), tiles[0].size() * sizeof(Tile));
    if (!tiles[1].empty()) std::memcpy(h + o_t1, tiles[1].data(), tiles[1].size() * sizeof(Tile));
    if (!cbc_groups.empty())
        std::memcpy(h + o_cg, cbc_groups.data(), cbc_groups.size() * sizeof(Tile));
    if (!cbc_list.empty())
        std::memcpy(h + o_cl, cbc_list.data(), cbc_list.size() * sizeof(uint32_t));

    DeviceGuard g(ctx->device);
    if (!g.ok()) return AESGPU_EHIP;
    uint8_t *d = static_cast<uint8_t *>(scratch_address(ctx->device));
    if (!d) return AESGPU_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // From pageable host memory, so the copy has read `staging` when the
    // call returns; it runs in stream order before the launches.
    if (hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, s) != hipSuccess) return AESGPU_EHIP;
    BatchLaunch L{};
    L.msgs = reinterpret_cast<const DevMsg *>(d + o_msgs);
    L.tiles[0] = reinterpret_cast<const Tile *>(d + o_t0);
    L.tiles[1] = reinterpret_cast<const Tile *>(d + o_t1);
    L.n_tiles[0] = uint32_t(tiles[0].size());
    L.n_tiles[1] = uint32_t(tiles[1].size());
    L.counters = reinterpret_cast<uint32_t *>(d);
    L.keys = d_keys;
    L.sched = nullptr;
    L.in = static_cast<const uint8_t *>(d_in);
    L.out = static_cast<uint8_t *>(d_out);
    L.tables = ctx->d_tables;
    L.cbc_list = reinterpret_cast<const uint32_t *>(d + o_cl);
    L.cbc_groups = reinterpret_cast<const Tile *>(d + o_cg);
    L.cbc_dummy = reinterpret_cast<uint4 *>(d + o_dummy);
    L.n_cbc_groups = uint32_t(cbc_groups.size());
    L.n_cu = ctx->n_cu;
    L.bpl = bpl;
    L.blocks[0] = tot.blocks[0];
    L.blocks[1] = tot.blocks[1];
    (void)use_graph;
    return enqueue_batch(L, s);
}

}  // extern "C"
