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
//  * Round keys are kernel arguments, so they are loaded once into SGPRs.
//  * 1024 threads per workgroup and one workgroup per CU (the tables take the
//    whole LDS); the grid is at most one workgroup per CU and strides over
//    tiles of 1024 * BPL blocks.
#include <hip/hip_runtime.h>

#include <cstdlib>

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
    uint32_t iv[4];
    CtrConsts cc;
    RoundKeys rk;
};

// Blocks base + j * kWG + threadIdx.x (j < BPL) that are below n_full; zero
// for the others.
template <int BPL>
__device__ __forceinline__ void load_tile(uint4 (&v)[BPL], const uint4 *in, uint64_t base,
                                          uint64_t n_full) {
#pragma unroll
    for (int j = 0; j < BPL; ++j) {
        const uint64_t idx = base + uint64_t(j) * kWG + threadIdx.x;
        v[j] = make_uint4(0, 0, 0, 0);
        if (idx < n_full) v[j] = in[idx];
    }
}

template <Op OP, int NR, int BPL>
__global__ __launch_bounds__(kWG) void aes_kernel(Params p) {
    constexpr bool kInv = (OP == Op::kEcbDec || OP == Op::kCbcDec);
    __shared__ uint32_t lds[kInv ? kFwdWords + kInvSWords : kFwdWords];
    stage_tables<kInv>(lds, p.tables);
    const Bases b = lane_bases();

    const uint64_t n_total = p.n_full + (p.tail ? 1 : 0);
    const uint64_t tile = uint64_t(kWG) * BPL;
    const uint64_t stride = uint64_t(gridDim.x) * tile;
    // The blocks of the next tile are loaded while the current one is
    // computed, so HBM latency overlaps the rounds even at low occupancy.
    uint4 next[BPL];
    load_tile<BPL>(next, p.in, uint64_t(blockIdx.x) * tile, p.n_full);
    for (uint64_t base = uint64_t(blockIdx.x) * tile; base < n_total; base += stride) {
        uint32_t s[BPL][4];
        uint4 in[BPL];
#pragma unroll
        for (int j = 0; j < BPL; ++j) in[j] = next[j];
        load_tile<BPL>(next, p.in, base + stride, p.n_full);
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            const uint64_t idx = base + uint64_t(j) * kWG + threadIdx.x;
            if constexpr (OP == Op::kEcbEnc || OP == Op::kEcbDec || OP == Op::kCbcDec) {
                s[j][0] = in[j].x ^ p.rk.w[0];
                s[j][1] = in[j].y ^ p.rk.w[1];
                s[j][2] = in[j].z ^ p.rk.w[2];
                s[j][3] = in[j].w ^ p.rk.w[3];
            } else if constexpr (OP == Op::kCtrBe32) {
                // Counter block: nonce words 0..2, word 3 = BE32(ctr0 + idx).
                // Round 1 is done here: output word c needs one lookup, on
                // byte (3 - c) of word 3; the other three terms are constants.
                const uint32_t w3 = bswap32(p.ctr0 + uint32_t(idx)) ^ p.cc.k03;
                s[j][0] = p.cc.p[0] ^ tlook<3>(lds, w3, b.t[3]);
                s[j][1] = p.cc.p[1] ^ tlook<2>(lds, w3, b.t[2]);
                s[j][2] = p.cc.p[2] ^ tlook<1>(lds, w3, b.t[1]);
                s[j][3] = p.cc.p[3] ^ tlook<0>(lds, w3, b.t[0]);
            } else {  // kCtrLe128: IV + index0 + idx as a 128-bit LE integer
                const uint64_t add = p.index0 + idx;
                const uint64_t lo0 = uint64_t(p.iv[0]) | (uint64_t(p.iv[1]) << 32);
                const uint64_t hi0 = uint64_t(p.iv[2]) | (uint64_t(p.iv[3]) << 32);
                const uint64_t lo = lo0 + add;
                const uint64_t hi = hi0 + (lo < lo0 ? 1u : 0u);
                s[j][0] = uint32_t(lo) ^ p.rk.w[0];
                s[j][1] = uint32_t(lo >> 32) ^ p.rk.w[1];
                s[j][2] = uint32_t(hi) ^ p.rk.w[2];
                s[j][3] = uint32_t(hi >> 32) ^ p.rk.w[3];
            }
        }
        const int first = (OP == Op::kCtrBe32) ? 2 : 1;
#pragma unroll
        for (int r = 1; r < NR; ++r) {
            if (r < first) continue;
#pragma unroll
            for (int j = 0; j < BPL; ++j) mid_round<kInv>(lds, b, s[j], &p.rk.w[4 * r]);
        }
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            if (kInv)
                last_round_inv(lds, b, s[j], &p.rk.w[4 * NR]);
            else
                last_round_fwd(lds, b, s[j], &p.rk.w[4 * NR]);
        }
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
            const uint64_t idx = base + uint64_t(j) * kWG + threadIdx.x;
            uint4 o = make_uint4(s[j][0], s[j][1], s[j][2], s[j][3]);
            if constexpr (OP == Op::kCtrBe32 || OP == Op::kCtrLe128) {
                o.x ^= in[j].x;
                o.y ^= in[j].y;
                o.z ^= in[j].z;
                o.w ^= in[j].w;
            } else if constexpr (OP == Op::kCbcDec) {
                // Eq. (2): XOR with the previous ciphertext block (IV first).
                uint4 prev = make_uint4(p.iv[0], p.iv[1], p.iv[2], p.iv[3]);
                if (idx > 0 && idx < p.n_full) prev = p.in[idx - 1];
                o.x ^= prev.x;
                o.y ^= prev.y;
                o.z ^= prev.z;
                o.w ^= prev.w;
            }
            if (idx < p.n_full) {
                p.out[idx] = o;
            } else if (idx == p.n_full && p.tail) {
                // Partial last block of a CTR call: byte-wise, only in range.
                const uint8_t *src = reinterpret_cast<const uint8_t *>(p.in + p.n_full);
                uint8_t *dst = reinterpret_cast<uint8_t *>(p.out + p.n_full);
                const uint32_t ks[4] = {s[j][0], s[j][1], s[j][2], s[j][3]};
                for (uint32_t q = 0; q < p.tail; ++q)
                    dst[q] = src[q] ^ uint8_t(ks[q >> 2] >> (8 * (q & 3)));
            }
        }
    }
}

template <Op OP, int NR, int BPL>
int launch_one(const Params &p, int n_cu, hipStream_t stream) {
    const uint64_t n_total = p.n_full + (p.tail ? 1 : 0);
    const uint64_t tiles = (n_total + uint64_t(kWG) * BPL - 1) / (uint64_t(kWG) * BPL);
    const uint32_t grid = uint32_t(tiles < uint64_t(n_cu) ? tiles : uint64_t(n_cu));
    hipLaunchKernelGGL((aes_kernel<OP, NR, BPL>), dim3(grid), dim3(kWG), 0, stream, p);
    return hipGetLastError() == hipSuccess ? AESGPU_OK : AESGPU_EHIP;
}

template <Op OP, int BPL>
int launch_nr(const Params &p, uint32_t nr, int n_cu, hipStream_t stream) {
    switch (nr) {
        case 10: return launch_one<OP, 10, BPL>(p, n_cu, stream);
        case 12: return launch_one<OP, 12, BPL>(p, n_cu, stream);
        case 14: return launch_one<OP, 14, BPL>(p, n_cu, stream);
        default: return AESGPU_EINVAL;
    }
}

template <Op OP>
int launch_op(const Params &p, uint32_t nr, int n_cu, hipStream_t stream) {
    static const int forced = [] {
        const char *e = std::getenv("AESGPU_FORCE_BPL");
        return e ? std::atoi(e) : 0;
    }();
    switch (forced) {
        case 1: return launch_nr<OP, 1>(p, nr, n_cu, stream);
        case 2: return launch_nr<OP, 2>(p, nr, n_cu, stream);
        default: return launch_nr<OP, 4>(p, nr, n_cu, stream);
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
    switch (a.op) {
        case Op::kEcbEnc: return launch_op<Op::kEcbEnc>(p, a.nr, n_cu, stream);
        case Op::kEcbDec: return launch_op<Op::kEcbDec>(p, a.nr, n_cu, stream);
        case Op::kCtrBe32: return launch_op<Op::kCtrBe32>(p, a.nr, n_cu, stream);
        case Op::kCtrLe128: return launch_op<Op::kCtrLe128>(p, a.nr, n_cu, stream);
        case Op::kCbcDec: return launch_op<Op::kCbcDec>(p, a.nr, n_cu, stream);
    }
    return AESGPU_EINVAL;
}

}  // namespace aesgpu
