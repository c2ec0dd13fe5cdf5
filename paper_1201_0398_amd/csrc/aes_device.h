// Device-side building blocks shared by the AES kernels: LDS table layout,
// table lookups, and the rounds of the paper's section 2.1 (Eq. (1)).
//
// LDS image (byte addresses; c = lane % 32 is the lane's private copy, so the
// bank of every lookup is fixed by the lane whatever the data):
//    T_t[x], copy c:      (t >> 1) * 65536 + x * 256 + (t & 1) * 128 + 4c   (128 KiB)
//    (InvS[x] | S[x]<<8): 131072 + x * 128 + 4c      (inverse set only, 32 KiB)
// The forward set holds T0..T3, the inverse set Td0..Td3 plus the S-box word.
// One v_perm_b32 forms a T address: byte k of the state word goes to bits
// 8..15 and the lane's per-table base supplies bits 0..7 and 16..23.
#pragma once

#include <hip/hip_runtime.h>

#include "aes_internal.h"

namespace aesgpu {
namespace dev {

constexpr int kWG = 1024;
constexpr uint32_t kFwdWords = 32768;      // replicated T0..T3 (or Td0..Td3)
constexpr uint32_t kInvSWords = 8192;      // replicated InvS
constexpr uint32_t kInvSByte = 4 * kFwdWords;


struct Bases {
    uint32_t t[4];  // byte address of this lane's copy of T_t[0]
    uint32_t invs;  // byte address of this lane's copy of InvS[0]
};

__device__ __forceinline__ Bases lane_bases() {
    const uint32_t c4 = (threadIdx.x & 31u) * 4u;
    return {{c4, c4 + 128u, c4 + 65536u, c4 + 65536u + 128u}, kInvSByte + c4};
}

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96 is symmetric in its inputs).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint32_t lds_at(const uint32_t *lds, uint32_t byte_addr) {
    return *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(lds) + byte_addr);
}

// T lookup indexed by byte K of `word`, in the table whose lane base is `base`.
template <int K>
__device__ __forceinline__ uint32_t tlook(const uint32_t *lds, uint32_t word, uint32_t base) {
    // v_perm_b32: result bytes {base.b0, word.bK, base.b2, 0}.
    const uint32_t addr = __builtin_amdgcn_perm(word, base, 0x0C020000u | ((4u + K) << 8));
    return lds_at(lds, addr);
}

// InvS lookup indexed by byte K of `word`: InvS in byte 0, S in byte 1.
template <int K>
__device__ __forceinline__ uint32_t islook(const uint32_t *lds, uint32_t word, uint32_t base) {
    const uint32_t x = (word >> (8 * K)) & 0xFFu;
    return lds_at(lds, (x << 7) + base);
}

// Byte 0 of v0, byte 1 of v1, byte 2 of v2 and byte 3 of v3, XORed with k.
// The two halves have disjoint bytes, so OR-ing them is the same as XOR.
__device__ __forceinline__ uint32_t merge4_xor(uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3,
                                               uint32_t k) {
    const uint32_t lo = __builtin_amdgcn_perm(v1, v0, 0x0C0C0500u);
    const uint32_t hi = __builtin_amdgcn_perm(v3, v2, 0x07020C0Cu);
    return xor3(lo, hi, k);
}

// Byte 0 of each of v0..v3 into bytes 0..3 of the result, XORed with k.
__device__ __forceinline__ uint32_t merge4_low_xor(uint32_t v0, uint32_t v1, uint32_t v2,
                                                   uint32_t v3, uint32_t k) {
    const uint32_t lo = __builtin_amdgcn_perm(v1, v0, 0x0C0C0400u);
    const uint32_t hi = __builtin_amdgcn_perm(v3, v2, 0x04000C0Cu);
    return xor3(lo, hi, k);
}

// One middle round, Eq. (1).  Forward: output word c reads byte k of word
// (c + k) mod 4.  Inverse (equivalent inverse cipher): word (c - k) mod 4.
template <bool kInv>
__device__ __forceinline__ void mid_round(const uint32_t *lds, const Bases &b, uint32_t (&s)[4],
                                          const uint32_t *k) {
    uint32_t o[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int i1 = kInv ? (c + 3) & 3 : (c + 1) & 3;
        const int i2 = (c + 2) & 3;
        const int i3 = kInv ? (c + 1) & 3 : (c + 3) & 3;
        o[c] = xor3(xor3(tlook<0>(lds, s[c], b.t[0]), tlook<1>(lds, s[i1], b.t[1]),
                         tlook<2>(lds, s[i2], b.t[2])),
                    tlook<3>(lds, s[i3], b.t[3]), k[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] = o[c];
}

// Last forward round: SubBytes + ShiftRows + AddRoundKey.  The S-box byte is
// taken from the T tables: T2 holds S(x) in byte 0, T3 in byte 1, T0 in byte
// 2 and T1 in byte 3.
__device__ __forceinline__ void last_round_fwd(const uint32_t *lds, const Bases &b,
                                               uint32_t (&s)[4], const uint32_t *k) {
    uint32_t o[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        o[c] = merge4_xor(tlook<0>(lds, s[c], b.t[2]), tlook<1>(lds, s[(c + 1) & 3], b.t[3]),
                          tlook<2>(lds, s[(c + 2) & 3], b.t[0]),
                          tlook<3>(lds, s[(c + 3) & 3], b.t[1]), k[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] = o[c];
}

// Last inverse round: InvSubBytes + InvShiftRows + AddRoundKey.
__device__ __forceinline__ void last_round_inv(const uint32_t *lds, const Bases &b,
                                               uint32_t (&s)[4], const uint32_t *k) {
    uint32_t o[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        o[c] = merge4_low_xor(islook<0>(lds, s[c], b.invs),
                              islook<1>(lds, s[(c + 3) & 3], b.invs),
                              islook<2>(lds, s[(c + 2) & 3], b.invs),
                              islook<3>(lds, s[(c + 1) & 3], b.invs), k[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] = o[c];
}

// Copies the table set into the LDS image; tid is the thread's index in the
// workgroup.  Loads are issued in groups of kGroup before their LDS writes, so
// the staging costs a few L2 round trips instead of one per word; a wave's
// loads hit two distinct words (every lane of a wave writes copies of the same
// table entry).  Needs blockDim.x == WG.
template <bool kInv, int WG = kWG, int kGroup = 16>
__device__ __forceinline__ void stage_tables_tid(uint32_t *lds, const uint32_t *__restrict__ g,
                                                 uint32_t tid) {
    static_assert(kFwdWords % (WG * kGroup) == 0 && kInvSWords % WG == 0, "workgroup size");
    const uint32_t *src = g + (kInv ? kTd : kTe);
    constexpr int kPer = kFwdWords / WG;
#pragma unroll 1
    for (int k0 = 0; k0 < kPer; k0 += kGroup) {
        uint32_t v[kGroup];
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            const uint32_t i = tid + uint32_t(k0 + k) * WG;
            const uint32_t t = ((i >> 14) << 1) | ((i >> 5) & 1u);
            const uint32_t x = (i >> 6) & 0xFFu;
            v[k] = src[t * 256u + x];
        }
#pragma unroll
        for (int k = 0; k < kGroup; ++k) lds[tid + uint32_t(k0 + k) * WG] = v[k];
    }
    if constexpr (kInv) {
        constexpr int kPerS = kInvSWords / WG;
#pragma unroll 1
        for (int k0 = 0; k0 < kPerS; k0 += 8) {
            uint32_t w[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                w[k] = k0 + k < kPerS ? g[kInvSS + ((tid + uint32_t(k0 + k) * WG) >> 5)] : 0u;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k0 + k < kPerS) lds[kFwdWords + tid + uint32_t(k0 + k) * WG] = w[k];
        }
    }
    __syncthreads();
}

template <bool kInv, int WG = kWG, int kGroup = 16>
__device__ __forceinline__ void stage_tables(uint32_t *lds, const uint32_t *__restrict__ g) {
    stage_tables_tid<kInv, WG, kGroup>(lds, g, threadIdx.x);
}

__device__ __forceinline__ uint32_t bswap32(uint32_t v) {
    return __builtin_amdgcn_perm(v, v, 0x00010203u);
}

// Raw buffer accesses.  The hardware checks each offset against the
// resource's range: past it a load reads zero and a store writes nothing.
// Kernels use them for block loads and stores so that no lane needs a branch
// and the compiler can count the outstanding memory operations exactly.
using rsrc_t = __amdgpu_buffer_rsrc_t;
using u32x4 = uint32_t __attribute__((ext_vector_type(4)));
constexpr int kRawBufferWord3 = 0x00020000;   // gfx9 raw buffer, 32-bit data format

__device__ __forceinline__ rsrc_t buffer_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, int(bytes),
                                             kRawBufferWord3);
}

__device__ __forceinline__ uint4 buffer_load16(rsrc_t r, uint32_t offset) {
    const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, offset, 0, 0);
    return make_uint4(x[0], x[1], x[2], x[3]);
}

__device__ __forceinline__ void buffer_store16(rsrc_t r, uint32_t offset, const uint4 &v) {
    const u32x4 x = {v.x, v.y, v.z, v.w};
    __builtin_amdgcn_raw_buffer_store_b128(x, r, offset, 0, 0);
}

// Pointers into the constant address space: a load through one with a
// wave-uniform address is a scalar load through the scalar cache.  Only for
// memory that no kernel in flight writes.
template <class T>
__device__ __forceinline__ const T __attribute__((address_space(4))) *as_const(const T *p) {
    return (const T __attribute__((address_space(4))) *)p;
}

}  // namespace dev
}  // namespace aesgpu
