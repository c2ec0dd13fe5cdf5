// gfx950 kernels for the T-table AES rounds (paper section 2.1, Eq. (1)) and
// the parallel modes of section 3: ECB both ways, CTR, CBC decryption.
//
// Design (CDNA4):
//  * One 16-byte block per lane per step, loaded and stored with one
//    global_load/store_dwordx4; a wave touches 1 KiB of contiguous HBM per
//    instruction.  Each lane carries BPL independent blocks for ILP.
//  * The four 1 KiB tables live in LDS, replicated 32 times so that lane L
//    always reads copy L % 32: the bank of every lookup is fixed by the lane,
//    whatever the data, so random table indices cause no bank conflicts.
//    Byte address of copy c of T_t[x]:
//        (t >> 1) * 65536 + x * 256 + (t & 1) * 128 + 4c          (128 KiB)
//    so one v_perm_b32 forms an address: byte k of the state word goes to
//    bits 8..15, the lane's per-table base supplies bits 0..7 and 16..23.
//  * Decryption adds InvS (replicated into all four bytes of a word) at
//    131072 + x * 128 + 4c, 32 KiB, for the last round: 160 KiB in total.
//  * Round keys are kernel arguments, so they are loaded once into SGPRs
//    (AES-256, AES-192 CTR and CBC: the middle rounds' keys from VGPRs).
//  * CTR (32-bit big-endian counter): wave w of a tile holds the 64 * BPL
//    consecutive blocks from 64 * BPL * w (slot j of lane L: block
//    64 * BPL * w + 64 * j + L), and the mapping is shifted by ctr0 mod
//    (64 * BPL) so that every wave holds 64 * BPL <= 256 consecutive counters
//    starting at a multiple of 64 * BPL.  Then only the low byte of
//    the counter differs across the wave: three of the four round-1 lookups
//    and twelve of the sixteen round-2 lookups have wave-uniform indices and
//    are read once per wave and tile through the scalar cache, leaving 5 LDS
//    lookups per block for the first two rounds.
//  * 1024 threads per workgroup and one workgroup per CU (the tables take the
//    whole LDS); the grid is at most one workgroup per CU and strides over
//    tiles of 1024 * BPL blocks.  BPL is 4 when every CU gets a full tile and
//    smaller for smaller buffers; at one block per lane a small buffer is cut
//    into tiles of 64..1024 blocks, one per CU.
//  * A tile is cut into 16 shares of 64 * BPL blocks, and a workgroup's waves
//    take the shares of its tiles in turn from a count in LDS, so that waves
//    the CU runs faster do more of them.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "aes_device.h"
#include "aes_internal.h"

namespace aesgpu {
namespace {

using namespace dev;

struct Params {
    const uint4 *in;
    uint4 *out;
    uint64_t n_full;        // whole blocks
    uint32_t tail;          // bytes of a final partial block (CTR only), 0..15
    uint32_t ctr0;
    const uint32_t *tables;
    uint64_t index0;        // LE-128 counter offset
    uint32_t ctr_y;         // LE-128: word 0 of the counter of virtual slot 0
    uint32_t voff;          // virtual index = block index + voff (CTR: ctr0 mod 64 * BPL)
    uint32_t tile;          // blocks per tile: kWG * BPL, or a multiple of 64 below kWG
                            // for small buffers at 1 block per lane
    uint32_t tiles_q;       // tiles in the launch, ceil((n_full + voff) / tile), divided by
    uint32_t tiles_r;       // the grid size: quotient and remainder
    uint32_t prev_in;       // CBC: 1 if block -1 (in[-1]) is ciphertext to chain from
                            // (a later part of a split call), 0 if block 0 takes the IV
    uint32_t iv[4];
    CtrConsts cc;
    RoundKeys rk;
};

// A tile of kWG * BPL blocks is cut into 16 shares of 64 * BPL blocks, one
// wave's work.  Position of slot j of this lane when its wave computes share w:
// slot-major (slot j of the tile is kWG consecutive blocks, share w its 64
// from 64 * w) or wave-major (share w is the 64 * BPL consecutive blocks from
// 64 * BPL * w, its slot j the 64 from 64 * j there).  Either way a wave's
// load or store instruction covers 64 consecutive blocks, 1 KiB.  (With each
// lane holding BPL consecutive blocks instead, an instruction touches 32 cache
// lines rather than 8: AES-128 ECB decryption ran 3% slower so.)
template <bool kWaveMajor, int BPL>
__device__ __forceinline__ uint32_t tile_slot(uint32_t w, int j) {
    const uint32_t lane = threadIdx.x & 63u;
    return kWaveMajor ? w * (64u * BPL) + uint32_t(j) * 64u + lane
                      : uint32_t(j) * kWG + w * 64u + lane;
}

// Lowest position of share w in its tile.
template <bool kWaveMajor, int BPL>
constexpr uint32_t kShareStep = kWaveMajor ? 64u * BPL : 64u;

// Buffer resources for the tile at virtual position base, so that every lane
// issues its loads and stores without a branch and the compiler can place
// the waits that let the next tile's loads overlap this tile's rounds.  The
// resource starts at the tile's first real block and covers the blocks of
// the tile that exist; lanes before block 0 get offsets that wrap to values
// far past any range.
struct TileView {
    rsrc_t in, out;
    uint32_t shift;   // lanes before block 0 in this tile (first tile only)
    uint32_t w;       // the share of the tile this wave computes
};

__device__ __forceinline__ TileView tile_view(const uint4 *in, uint4 *out, uint64_t base,
                                              uint32_t w, uint64_t n_full, uint32_t voff,
                                              uint32_t tile) {
    const uint64_t first = base >= voff ? base - voff : 0;
    const uint32_t shift = base >= voff ? 0u : voff;
    const uint64_t left = first < n_full ? n_full - first : 0;
    const uint32_t bytes = 16u * uint32_t(left < tile ? left : tile);
    return {buffer_rsrc(in + first, bytes), buffer_rsrc(out + first, bytes), shift, w};
}

template <bool kWaveMajor, int BPL>
__device__ __forceinline__ uint32_t lane_offset(const TileView &v, int j) {
    return (tile_slot<kWaveMajor, BPL>(v.w, j) - v.shift) * 16u;
}

template <bool kWaveMajor, int BPL>
__device__ __forceinline__ void load_tile(uint4 (&v)[BPL], const TileView &t) {
#pragma unroll
    for (int j = 0; j < BPL; ++j) v[j] = buffer_load16(t.in, lane_offset<kWaveMajor, BPL>(t, j));
}

template <bool kWaveMajor, int BPL>
__device__ __forceinline__ void store_block(const TileView &t, int j, const uint4 &o) {
    buffer_store16(t.out, lane_offset<kWaveMajor, BPL>(t, j), o);
}

// The next share for this wave: lane 0 adds one to the workgroup's count in
// LDS and the old count goes to every lane.  The exec mask is narrowed inside
// the asm block, which also waits for the result, so the tile loop has no
// branch.  The count is kept in the high half of its word (in decryption
// kernels the low half holds an InvS table entry, which the add leaves as it
// is).  Needs all 64 lanes of the wave active.  No memory clobber: the only
// LDS data the add shares a word with is read-only, and with the clobber the
// compiler kept only about five table reads in flight in AES-256 encryption.
__device__ __forceinline__ uint32_t claim_share(uint32_t *count) {
    uint32_t old = 0;
    uint64_t exec_save;
    const uint32_t addr = uint32_t(reinterpret_cast<uintptr_t>(count));   // LDS offset
    asm volatile(
        "s_mov_b64 %1, exec\n\t"
        "s_mov_b64 exec, 1\n\t"
        "ds_add_rtn_u32 %0, %2, %3\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "s_mov_b64 exec, %1\n\t"
        "s_nop 4"
        : "+v"(old), "=&s"(exec_save)
        : "v"(addr), "v"(0x10000u));
    return uint32_t(__builtin_amdgcn_readfirstlane(old)) >> 16;
}

// Lane L gets x of lane L - 1 (a DPP shift of the wave); lane 0 keeps lane0.
__device__ __forceinline__ uint4 from_lane_below(const uint4 &lane0, const uint4 &x) {
    return make_uint4(__builtin_amdgcn_update_dpp(lane0.x, x.x, 0x138, 0xf, 0xf, false),
                      __builtin_amdgcn_update_dpp(lane0.y, x.y, 0x138, 0xf, 0xf, false),
                      __builtin_amdgcn_update_dpp(lane0.z, x.z, 0x138, 0xf, 0xf, false),
                      __builtin_amdgcn_update_dpp(lane0.w, x.w, 0x138, 0xf, 0xf, false));
}

// Lane 0 gets x of lane 63 (a DPP rotation of the wave; the other lanes get
// lane L - 1's, which from_lane_below then replaces).
__device__ __forceinline__ uint4 from_lane_63(const uint4 &x) {
    return make_uint4(__builtin_amdgcn_mov_dpp(x.x, 0x13C, 0xf, 0xf, false),
                      __builtin_amdgcn_mov_dpp(x.y, 0x13C, 0xf, 0xf, false),
                      __builtin_amdgcn_mov_dpp(x.z, 0x13C, 0xf, 0xf, false),
                      __builtin_amdgcn_mov_dpp(x.w, 0x13C, 0xf, 0xf, false));
}

// CBC (wave-major tiles): block first - 1, where first = base + 64 * BPL * w
// is the first block of share w of the tile at base (the same address in
// every lane), read through a resource that starts one block before the tile;
// zero past the end, and where first == 0 unless block -1 exists (prev_in; if
// not, the caller substitutes the IV).
template <int BPL>
__device__ __forceinline__ uint4 load_wave_prev(const uint4 *in, uint64_t base, uint32_t w,
                                                uint64_t n_full, uint32_t tile, uint32_t prev_in) {
    const bool before = base > 0 || prev_in;
    const uint32_t shift = before ? 0u : 1u;
    // The resource is the same in every lane; the compiler does not see that
    // through the select and would otherwise load in a loop over lane values.
    const uint64_t at = reinterpret_cast<uint64_t>(in + base) - 16u * (1u - shift);
    const uint64_t left = base < n_full ? n_full - base + 1 - shift : 0;
    const uint32_t bytes = 16u * uint32_t(left < tile + 1u ? left : tile + 1u);
    // (readfirstlane returns an int: each half is taken as unsigned before it
    // is widened, or a low word with bit 31 set would fill the high word.)
    const uint64_t at_u = uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(at)))) |
                          (uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(at >> 32)))) << 32);
    const rsrc_t r = buffer_rsrc(reinterpret_cast<const void *>(at_u),
                                 uint32_t(__builtin_amdgcn_readfirstlane(bytes)));
    return buffer_load16(r, (w * 64u * BPL - shift) * 16u);
}

// T_t[x] from the table copy in device memory, for an index that is the same
// in every lane: one scalar load instead of an LDS instruction.
__device__ __forceinline__ uint32_t tab_u(const uint32_t *te, uint32_t t, uint32_t x) {
    return as_const(te)[__builtin_amdgcn_readfirstlane(t * 256u + x)];
}

__device__ __forceinline__ uint32_t byte_of(uint32_t w, int k) { return (w >> (8 * k)) & 0xFFu; }

// Whitened counter block (round 0 done) of block idx for the CTR modes.
template <Op OP>
__device__ __forceinline__ void counter_state(const Params &p, uint64_t idx, uint32_t (&s)[4]) {
    if constexpr (OP == Op::kCtrBe32) {
        // nonce words 0..2, word 3 = BE32(ctr0 + idx)
        s[0] = p.cc.x0[0];
        s[1] = p.cc.x0[1];
        s[2] = p.cc.x0[2];
        s[3] = bswap32(p.ctr0 + uint32_t(idx)) ^ p.cc.kvar;
    } else {
        // IV + index0 + idx as a 128-bit little-endian integer
        const uint64_t add = p.index0 + idx;
        const uint64_t lo0 = uint64_t(p.iv[0]) | (uint64_t(p.iv[1]) << 32);
        const uint64_t hi0 = uint64_t(p.iv[2]) | (uint64_t(p.iv[3]) << 32);
        const uint64_t lo = lo0 + add;
        const uint64_t hi = hi0 + (lo < lo0 ? 1u : 0u);
        s[0] = uint32_t(lo) ^ p.rk.w[0];
        s[1] = uint32_t(lo >> 32) ^ p.rk.w[1];
        s[2] = uint32_t(hi) ^ p.rk.w[2];
        s[3] = uint32_t(hi >> 32) ^ p.rk.w[3];
    }
}

template <int I>
__device__ __forceinline__ uint32_t row_word(uint32_t x) {
    return uint32_t(__builtin_amdgcn_mov_dpp(int(x), 0x150 + I, 0xf, 0xf, false));
}

// Middle rounds R .. NR - 1, round keys from kq by row broadcast: kq[x], lane
// i of every row, holds word i % 4 of round 4x + 1 + i / 4.
template <bool kInv, int BPL, int R, int NR>
__device__ __forceinline__ void rounds_v(const uint32_t *lds, const Bases &b, uint32_t (&s)[BPL][4],
                                         const uint32_t (&kq)[4]) {
    if constexpr (R < NR) {
        constexpr int kX = (R - 1) / 4, kI = 4 * ((R - 1) % 4);
        const uint32_t k[4] = {row_word<kI>(kq[kX]), row_word<kI + 1>(kq[kX]),
                               row_word<kI + 2>(kq[kX]), row_word<kI + 3>(kq[kX])};
#pragma unroll
        for (int j = 0; j < BPL; ++j) mid_round<kInv>(lds, b, s[j], k);
        rounds_v<kInv, BPL, R + 1, NR>(lds, b, s, kq);
    }
}

// kDyn: the waves claim the shares of the workgroup's tiles from a count in
// LDS (launches with several tiles per CU); otherwise wave i computes share i
// of each of the workgroup's tiles.
template <Op OP, int NR, int BPL, bool kDyn>
__global__ __launch_bounds__(kWG) void aes_kernel(Params p) {
    constexpr bool kInv = (OP == Op::kEcbDec || OP == Op::kCbcDec);
    constexpr bool kCtr = (OP == Op::kCtrBe32 || OP == Op::kCtrLe128);
    constexpr bool kWM = kCtr || OP == Op::kCbcDec;   // wave-major tiles
    // The workgroup's share count: the word after the forward tables, which
    // in decryption kernels is the first copy of InvS[0] (its high half is
    // zero after the staging; the InvS entry uses bytes 0 and 1).
    __shared__ uint32_t lds[kInv ? kFwdWords + kInvSWords : kFwdWords + (kDyn ? 1 : 0)];
    uint32_t *const count = lds + kFwdWords;
    // Odd waves issue at a higher priority than even ones (a workgroup's
    // waves go to the CU's four SIMDs in turn, so two SIMDs run high and two
    // low).  The halves then drift out of step: one half's rounds issue table
    // reads while the other's XOR, and the LDS idles less.  Measured on
    // AES-128 ECB at 1 GiB: 1.5-2% faster than equal priorities (interleaved
    // runs); four priority levels, or a split by workgroup half, gained less.
    if ((threadIdx.x >> 6) & 1u) __builtin_amdgcn_s_setprio(2);

    // The loop covers the whole blocks; a CTR tail is finished after it.
    const uint64_t v_end = p.n_full ? p.n_full + p.voff : 0;
    const uint64_t tile = p.tile;
    const uint64_t stride = uint64_t(gridDim.x) * tile;
    // The workgroup's tiles (blockIdx.x, then every gridDim.x-th) are cut into
    // 16 shares each, numbered in order: share c is share c % 16 of tile
    // c / 16.  Wave i takes share i first; with kDyn the waves then claim
    // the next shares from the count as they finish, so fast waves take more:
    // the CU's arbitration gives its waves very unequal rates (with a fixed
    // share per wave, the last wave of a workgroup ended up to 2.4 times
    // later than its first), and claiming evens the waves' end times out.
    // A share exists if its first position is before the end; shares are
    // numbered in position order, so the workgroup's shares are 0 .. n_shares
    // - 1 and a wave's first claim past them is its last.  With at most
    // 16 * kMaxTilesPerCu shares, the 16-bit count never wraps.
    auto tile_of = [&](uint32_t c) -> uint64_t {
        return uint64_t(blockIdx.x) * tile + uint64_t(c >> 4) * stride;
    };
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t cur = wave;
    // The blocks of the next share are loaded while the current one is
    // computed, so HBM latency overlaps the rounds even at low occupancy.
    // The first share's loads are issued before the tables are staged, so
    // their HBM latency overlaps the staging.
    uint4 next[BPL];
    uint4 next_prev = make_uint4(0, 0, 0, 0);   // CBC only
    TileView view = tile_view(p.in, p.out, tile_of(cur), cur & 15u, p.n_full, p.voff, tile);
    load_tile<kWM, BPL>(next, view);
    if constexpr (OP == Op::kCbcDec) {
        // (Launches with one share per wave never chain from block -1, and
        // with prev_in known to be 0 the compiler kept twice as many table
        // reads in flight in AES-128 CBC at one block per lane.)
        next_prev = load_wave_prev<BPL>(p.in, tile_of(cur), cur & 15u, p.n_full, uint32_t(tile),
                                        kDyn ? p.prev_in : 0u);
        // Block 0 is the first block of share 0 of workgroup 0, which wave 0
        // takes first: its predecessor, the IV, is put in here rather than
        // chosen in the loop.  (Chosen there, it put a branch in the loop and
        // kept four more SGPRs live, and the compiler kept only ≈5 table reads
        // in flight per wave instead of ≈17.)
        if (blockIdx.x == 0 && cur == 0 && !(kDyn && p.prev_in))
            next_prev = make_uint4(p.iv[0], p.iv[1], p.iv[2], p.iv[3]);
    }
    // The share count is worked out after the first loads are issued, and its
    // kernel arguments are read with theirs: placed before the loads, or read
    // after the staging, it cost a second round trip for kernel arguments and
    // a small call (one tile per CU) about 1.3 us.
    uint32_t n_tiles_wg = p.tiles_q + (blockIdx.x < p.tiles_r ? 1u : 0u);
    if constexpr (kDyn) {
        asm volatile("" : "+s"(n_tiles_wg));
        if constexpr (!kInv)
            if (threadIdx.x == 0) *count = 0u;   // published by the staging barrier
    }
    stage_tables<kInv>(lds, p.tables);
    constexpr uint32_t kStep = kShareStep<kWM, BPL>;
    uint32_t n_shares = 0;
    if constexpr (kDyn) {
        if (n_tiles_wg) {
            const uint64_t left = v_end - tile_of((n_tiles_wg - 1u) << 4);   // > 0
            n_shares = (n_tiles_wg - 1u) * 16u +
                       uint32_t(std::min<uint64_t>(16, (left + kStep - 1) / kStep));
        }
    } else {
        // A small tile leaves the workgroup's last waves without blocks: they
        // end here (the staging barrier was the last one).
        if (wave * kStep >= p.tile) return;
    }
    const Bases b = lane_bases();
    // AES-256, and AES-192 CTR and CBC, take their middle rounds' keys from
    // VGPRs by row broadcast (DPP) rather than holding all of them in SGPRs:
    // with the SGPRs near their limit the compiler keeps only 3-4 table reads
    // in flight per wave (about 16 otherwise), and these kernels ran 6-8%
    // slower.  kq[x], lane i of every row of 16, holds word i % 4 of round
    // 4x + 1 + i / 4.
    constexpr bool kKeysV = NR == 14 || ((kCtr || OP == Op::kCbcDec) && NR == 12);
    uint32_t kq[4] = {0, 0, 0, 0};
    if constexpr (kKeysV) {
        const uint32_t l15 = threadIdx.x & 15u;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            uint32_t v = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int w = 4 * (4 * x + 1) + i;
                if (w < 4 * (NR + 1)) v = l15 == uint32_t(i) ? p.rk.w[w] : v;
            }
            kq[x] = v;
            asm volatile("" : "+v"(kq[x]));   // a VGPR value from here on
        }
    }
    // In the loop a tile's loads are followed by the previous tile's stores,
    // and the loop top waits for the loads only.  These stores have an empty
    // range and write nothing; they give the loop entry the same order, so
    // that wait does not also cover the last stores on every iteration.
    {
        const rsrc_t none = buffer_rsrc(p.out, 0);
#pragma unroll
        for (int j = 0; j < BPL; ++j)
            buffer_store16(none, lane_offset<kWM, BPL>(view, j), make_uint4(0, 0, 0, 0));
    }
    // One step: share w of the tile at base, while the blocks of share
    // next_w of the tile at next_base are loaded.
    auto step = [&](uint64_t base, uint32_t w, uint64_t next_base, uint32_t next_w) {
        uint32_t s[BPL][4];
        uint4 in[BPL];
#pragma unroll
        for (int j = 0; j < BPL; ++j) in[j] = next[j];
        const uint4 wave_prev = next_prev;
        const TileView now = view;
        view = tile_view(p.in, p.out, next_base, next_w, p.n_full, p.voff, tile);
        load_tile<kWM, BPL>(next, view);
        if constexpr (OP == Op::kCbcDec)
            next_prev = load_wave_prev<BPL>(p.in, next_base, next_w, p.n_full, uint32_t(tile),
                                            kDyn ? p.prev_in : 0u);
        // CTR rounds 1 and 2.  The wave's 64 * BPL counters start at a
        // multiple of 64 * BPL, so they differ only in their low byte, and so
        // does the whitened counter block.  Round 1 (Eq. (1)): the varying
        // byte feeds one table term of output word 0; the other 15 terms and
        // output words 1..3 are wave-uniform.  Round 2: each output word has
        // one term on word 0 (per block) and three on words 1..3 (uniform).
        // The uniform lookups are scalar loads, once per wave and tile.
        uint32_t c[4] = {0, 0, 0, 0};   // round-2 uniform part, per output word
        uint32_t r1 = 0;                // round-1 uniform part of word 0
        uint32_t y0 = 0;                // LE-128: counter word 0 of the wave's first slot
        uint32_t w3u = 0;               // BE32: whitened word 3 of the wave's first counter
        if constexpr (kCtr) {
            const uint32_t *te = p.tables + kTe;
            uint32_t u1, u2, u3;        // round-1 output words 1..3
            if constexpr (OP == Op::kCtrBe32) {
                // Counter block: nonce words 0..2 (folded into cc.p by the
                // host), word 3 = BE32(counter), whose byte 3 varies.
                const uint32_t ctr_first = p.ctr0 - p.voff + uint32_t(base) + w * (64u * BPL);
                w3u = bswap32(ctr_first) ^ p.cc.kvar;
                r1 = p.cc.p[0];
                u1 = p.cc.p[1] ^ tab_u(te, 2, byte_of(w3u, 2));
                u2 = p.cc.p[2] ^ tab_u(te, 1, byte_of(w3u, 1));
                u3 = p.cc.p[3] ^ tab_u(te, 0, byte_of(w3u, 0));
            } else {
                // Counter block: the 128-bit LE integer whose words 1..3 are
                // fixed over the launch (folded into cc.p by the host) and
                // whose word 0 is ctr_y + slot; its byte 0 varies.
                y0 = p.ctr_y + uint32_t(base) + w * (64u * BPL);
                const uint32_t s0u = y0 ^ p.cc.kvar;
                r1 = p.cc.p[0];
                u1 = p.cc.p[1] ^ tab_u(te, 3, byte_of(s0u, 3));
                u2 = p.cc.p[2] ^ tab_u(te, 2, byte_of(s0u, 2));
                u3 = p.cc.p[3] ^ tab_u(te, 1, byte_of(s0u, 1));
            }
            const uint32_t *k2 = &p.rk.w[8];
            c[0] = tab_u(te, 1, byte_of(u1, 1)) ^ tab_u(te, 2, byte_of(u2, 2)) ^
                   tab_u(te, 3, byte_of(u3, 3)) ^ k2[0];
            c[1] = tab_u(te, 0, byte_of(u1, 0)) ^ tab_u(te, 1, byte_of(u2, 1)) ^
                   tab_u(te, 2, byte_of(u3, 2)) ^ k2[1];
            c[2] = tab_u(te, 0, byte_of(u2, 0)) ^ tab_u(te, 1, byte_of(u3, 1)) ^
                   tab_u(te, 3, byte_of(u1, 3)) ^ k2[2];
            c[3] = tab_u(te, 0, byte_of(u3, 0)) ^ tab_u(te, 2, byte_of(u1, 2)) ^
                   tab_u(te, 3, byte_of(u2, 3)) ^ k2[3];
        }
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            if constexpr (OP == Op::kEcbEnc || OP == Op::kEcbDec || OP == Op::kCbcDec) {
                s[j][0] = in[j].x ^ p.rk.w[0];
                s[j][1] = in[j].y ^ p.rk.w[1];
                s[j][2] = in[j].z ^ p.rk.w[2];
                s[j][3] = in[j].w ^ p.rk.w[3];
            } else {
                // Round-1 word 0: the one per-block lookup of round 1.
                uint32_t v0;
                if constexpr (OP == Op::kCtrBe32) {
                    // Slot j of lane L has counter ctr_first + 64 j + L, and
                    // ctr_first is a multiple of 64 * BPL > 64 j + L: the sum
                    // only sets low bits of the counter's low byte, which is
                    // byte 3 of the big-endian word.
                    const uint32_t w3 = w3u ^ ((uint32_t(j) * 64u + (threadIdx.x & 63u)) << 24);
                    v0 = r1 ^ tlook<3>(lds, w3, b.t[3]);
                } else {
                    const uint32_t w0 = (y0 | (uint32_t(j) * 64u + (threadIdx.x & 63u))) ^ p.cc.kvar;
                    v0 = r1 ^ tlook<0>(lds, w0, b.t[0]);
                }
                s[j][0] = tlook<0>(lds, v0, b.t[0]) ^ c[0];
                s[j][1] = tlook<3>(lds, v0, b.t[3]) ^ c[1];
                s[j][2] = tlook<2>(lds, v0, b.t[2]) ^ c[2];
                s[j][3] = tlook<1>(lds, v0, b.t[1]) ^ c[3];
            }
        }
        const int first = kCtr ? 3 : 1;
#pragma unroll
        for (int r = 1; r < NR; ++r) {
            if (r < first) continue;
            if constexpr (!kKeysV) {
#pragma unroll
                for (int j = 0; j < BPL; ++j) mid_round<kInv>(lds, b, s[j], &p.rk.w[4 * r]);
            }
        }
        if constexpr (kKeysV) rounds_v<kInv, BPL, (kCtr ? 3 : 1), NR>(lds, b, s, kq);
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            if (kInv)
                last_round_inv(lds, b, s[j], &p.rk.w[4 * NR]);
            else
                last_round_fwd(lds, b, s[j], &p.rk.w[4 * NR]);
        }
        if constexpr (OP == Op::kCbcDec) {
            // Keeps the wave shuffles of the ciphertext below (DPP) after the
            // last round's table reads: placed among the rounds, they held 16
            // more VGPRs there and the compiler kept fewer reads in flight.
#pragma unroll
            for (int j = 0; j < BPL; ++j)
                asm volatile("" : "+v"(in[j].x), "+v"(in[j].y), "+v"(in[j].z), "+v"(in[j].w));
        }
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            uint4 o = make_uint4(s[j][0], s[j][1], s[j][2], s[j][3]);
            if constexpr (kCtr) {
                o.x ^= in[j].x;
                o.y ^= in[j].y;
                o.z ^= in[j].z;
                o.w ^= in[j].w;
            } else if constexpr (OP == Op::kCbcDec) {
                // Eq. (2): XOR with the previous ciphertext block: slot j of
                // lane L - 1; for lane 0, slot j - 1 of lane 63, or for slot 0
                // the block loaded with the tile (the IV for block 0, set
                // before the loop).
                const uint4 q = from_lane_below(j > 0 ? from_lane_63(in[j > 0 ? j - 1 : 0]) : wave_prev,
                                                in[j]);
                o.x ^= q.x;
                o.y ^= q.y;
                o.z ^= q.z;
                o.w ^= q.w;
            }
            store_block<kWM, BPL>(now, j, o);
        }
    };
    // The shares of a partial last tile with no block are not computed: a
    // partial tile of a few blocks otherwise costs a whole tile's rounds.
    if constexpr (kDyn) {
        while (cur < n_shares) {
            const uint64_t base = tile_of(cur);
            const uint32_t w = cur & 15u;
            cur = 16u + claim_share(count);
            step(base, w, tile_of(cur), cur & 15u);
        }
    } else {
        // A wave leaves the loop at the first tile that has no block for it.
        for (uint64_t base = uint64_t(blockIdx.x) * tile; base + uint64_t(wave) * kStep < v_end;
             base += stride)
            step(base, wave, base + stride, wave);
    }
    if constexpr (kCtr) {
        // Partial last block: wave 0 of workgroup 0 computes its keystream
        // (the same block in every lane) and lane q < tail writes byte q.
        if (p.tail && blockIdx.x == 0 && threadIdx.x < 64) {
            uint32_t s[4];
            counter_state<OP>(p, p.n_full, s);
#pragma unroll
            for (int r = 1; r < NR; ++r) mid_round<false>(lds, b, s, &p.rk.w[4 * r]);
            last_round_fwd(lds, b, s, &p.rk.w[4 * NR]);
            const uint32_t q = threadIdx.x;
            if (q < p.tail) {
                const uint8_t *src = reinterpret_cast<const uint8_t *>(p.in + p.n_full);
                uint8_t *dst = reinterpret_cast<uint8_t *>(p.out + p.n_full);
                const uint32_t w = q < 4 ? s[0] : q < 8 ? s[1] : q < 12 ? s[2] : s[3];
                dst[q] = src[q] ^ uint8_t(w >> (8 * (q & 3)));
            }
        }
    }
}

template <Op OP, int NR, int BPL>
int launch_part(Params p, int n_cu, hipStream_t stream) {
    // CTR: shift the mapping so every wave's 64 * BPL counters start at a
    // multiple of 64 * BPL (so they differ only in their low byte).
    if constexpr (OP == Op::kCtrBe32) {
        p.voff = p.ctr0 & (64u * BPL - 1u);
    } else if constexpr (OP == Op::kCtrLe128) {
        // Word 0 of the counter of block 0 is iv[0] + index0 (words 1..3 are
        // fixed over the launch; the host splits calls where word 0 wraps).
        const uint32_t x0 = p.iv[0] + uint32_t(p.index0);
        p.voff = x0 & (64u * BPL - 1u);
        p.ctr_y = x0 - p.voff;
    } else {
        p.voff = 0;
    }
    // At least one workgroup: a CTR call shorter than a block has only a tail.
    const uint64_t v_end = p.n_full ? p.n_full + p.voff : 0;
    // Tiles of kWG * BPL blocks; at one block per lane (small buffers) the
    // blocks are spread over every CU instead, in tiles of a multiple of 64
    // blocks (whole waves): a small call then costs the table staging and a
    // few waves' rounds per CU rather than a whole 1024-block tile on a few.
    uint64_t tile = uint64_t(kWG) * BPL;
    if (BPL == 1) {
        const uint64_t per_cu = (v_end + uint64_t(n_cu) - 1) / uint64_t(n_cu);
        tile = std::min<uint64_t>(kWG, std::max<uint64_t>(64, (per_cu + 63) & ~uint64_t(63)));
    }
    p.tile = uint32_t(tile);
    const uint64_t tiles = (v_end + tile - 1) / tile;
    const uint32_t grid = tiles == 0 ? 1u : uint32_t(tiles < uint64_t(n_cu) ? tiles : uint64_t(n_cu));
    p.tiles_q = uint32_t(tiles / grid);
    p.tiles_r = uint32_t(tiles % grid);
    // With at most one tile per CU the waves have nothing to even out, and a
    // small call ran about 1.2 us longer with the share count (measured at
    // 16 KiB .. 1 MiB; at 4 MiB, one tile of 1024 blocks per CU, both took
    // the same time): such launches at one block per lane keep one share per
    // wave, unless they are a later part of a split CBC call.
    const void *kernel = reinterpret_cast<const void *>(&aes_kernel<OP, NR, BPL, true>);
    if constexpr (BPL == 1)
        if (tiles <= uint64_t(n_cu) && !p.prev_in)
            kernel = reinterpret_cast<const void *>(&aes_kernel<OP, NR, BPL, false>);
    // The launch's own status (the thread's last-error state may hold an
    // earlier, unrelated failure).
    void *args[] = {&p};
    return hipLaunchKernel(kernel, dim3(grid), dim3(kWG), args, 0, stream) == hipSuccess
               ? AESGPU_OK
               : AESGPU_EHIP;
}

// Launches in parts of at most max_tiles - 1 tiles of kWG * BPL blocks per CU,
// so that a workgroup has at most max_tiles tiles (one more for the CTR shift)
// and 16 * max_tiles shares.  A part is a whole number of tiles, so the CTR
// shift is the same in every part; a later CBC part chains from the block
// before it, and only the last part has the CTR tail.
template <Op OP, int NR, int BPL>
int launch_one(const Params &p, int n_cu, uint32_t max_tiles, hipStream_t stream) {
    const uint64_t part = uint64_t(max_tiles - 1) * uint64_t(n_cu) * uint64_t(kWG) * BPL;
    Params q = p;
    for (uint64_t done = 0;; done += part) {
        const bool last = p.n_full - done <= part;
        q.in = p.in + done;
        q.out = p.out + done;
        q.n_full = last ? p.n_full - done : part;
        q.tail = last ? p.tail : 0u;
        q.ctr0 = p.ctr0 + uint32_t(done);
        q.index0 = p.index0 + done;
        q.prev_in = done > 0 ? 1u : p.prev_in;
        const int st = launch_part<OP, NR, BPL>(q, n_cu, stream);
        if (st != AESGPU_OK || last) return st;
    }
}

template <Op OP, int BPL>
int launch_nr(const Params &p, uint32_t nr, int n_cu, uint32_t max_tiles, hipStream_t stream) {
    switch (nr) {
        case 10: return launch_one<OP, 10, BPL>(p, n_cu, max_tiles, stream);
        case 12: return launch_one<OP, 12, BPL>(p, n_cu, max_tiles, stream);
        case 14: return launch_one<OP, 14, BPL>(p, n_cu, max_tiles, stream);
        default: return AESGPU_EINVAL;
    }
}

template <Op OP>
int launch_op(const Params &p, uint32_t nr, int n_cu, int forced_bpl, uint32_t max_tiles,
              hipStream_t stream) {
    int bpl = forced_bpl;
    if (bpl != 1 && bpl != 2 && bpl != 4) {
        // Every lane computes all its slots, empty or not, and a workgroup
        // overlaps a tile's rounds with the next tile's loads only when it has
        // several tiles.  Measured on AES-128 ECB encryption (µs per call,
        // 1 / 2 / 4 blocks per lane): 24 MiB 20.6 / 21.3 / 26.9, 64 MiB
        // 46.6 / 46.7 / 48.0, 128 MiB 89.4 / 89.1 / 89.9, 192 MiB
        // 142.1 / 142.3 / 140.6, 1 GiB 743 / 733 / 725.  So 4 blocks per lane
        // once every CU gets 12 tiles of 4096 blocks, 2 once it gets 16 tiles
        // of 2048, 1 below (at 1, small buffers are cut into smaller tiles).
        const uint64_t blocks = p.n_full + (p.tail ? 1 : 0);
        const uint64_t per_cu = (blocks + uint64_t(n_cu) - 1) / uint64_t(n_cu);
        bpl = per_cu >= 12ull * kWG * 4 ? 4 : per_cu >= 16ull * kWG * 2 ? 2 : 1;
        // CBC decryption with AES-192 or AES-256 keys at 4 blocks per lane
        // runs out of VGPRs (it keeps the ciphertext for the XOR of Eq. (2))
        // and spills in its loop; at 2 blocks per lane it ran 1.7-2.1% faster
        // at 1 GiB.
        if (OP == Op::kCbcDec && nr >= 12 && bpl == 4) bpl = 2;
    }
    switch (bpl) {
        case 1: return launch_nr<OP, 1>(p, nr, n_cu, max_tiles, stream);
        case 2: return launch_nr<OP, 2>(p, nr, n_cu, max_tiles, stream);
        default: return launch_nr<OP, 4>(p, nr, n_cu, max_tiles, stream);
    }
}

}  // namespace

int launch(const uint32_t *d_tables, int n_cu, const LaunchArgs &a, hipStream_t stream) {
    Params p{};
    p.in = static_cast<const uint4 *>(a.in);
    p.out = static_cast<uint4 *>(a.out);
    p.n_full = a.n_bytes / 16;
    p.tail = uint32_t(a.n_bytes % 16);
    p.ctr0 = a.ctr0;
    p.tables = d_tables;
    p.index0 = a.index0;
    for (int i = 0; i < 4; ++i) p.iv[i] = a.iv[i];
    p.cc = a.ctr;
    p.rk = *a.rk;
    const uint32_t mt = a.max_tiles >= 2 && a.max_tiles <= kMaxTilesPerCu ? a.max_tiles
                                                                          : kMaxTilesPerCu;
    switch (a.op) {
        case Op::kEcbEnc: return launch_op<Op::kEcbEnc>(p, a.nr, n_cu, a.bpl, mt, stream);
        case Op::kEcbDec: return launch_op<Op::kEcbDec>(p, a.nr, n_cu, a.bpl, mt, stream);
        case Op::kCtrBe32: return launch_op<Op::kCtrBe32>(p, a.nr, n_cu, a.bpl, mt, stream);
        case Op::kCtrLe128: return launch_op<Op::kCtrLe128>(p, a.nr, n_cu, a.bpl, mt, stream);
        case Op::kCbcDec: return launch_op<Op::kCbcDec>(p, a.nr, n_cu, a.bpl, mt, stream);
    }
    return AESGPU_EINVAL;
}

}  // namespace aesgpu
