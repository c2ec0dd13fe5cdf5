// Internal declarations shared by the host runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "aesgpu.h"

namespace aesgpu {

// Device table image, in 32-bit words, uploaded once per context:
//   [kTe + 256*k + x]  T_k[x]  = column MixColumns makes from S(x) in row k
//   [kTd + 256*k + x]  Td_k[x] = column InvMixColumns makes from InvS(x) in row k
//   [kInvSS + x]       InvS(x) in byte 0 and S(x) in byte 1
constexpr int kTe = 0;
constexpr int kTd = 1024;
constexpr int kInvSS = 2048;

constexpr int kTableWords = 2304;

// Round keys as kernel arguments: 15 rounds x 4 little-endian words.
struct alignas(16) RoundKeys {
    uint32_t w[60];
};

// First-round constants of the CTR modes.  Three of the four counter words
// are fixed over a launch (the nonce for the 32-bit big-endian counter, words
// 1..3 of the 128-bit little-endian counter, which the host keeps fixed by
// splitting a call where word 0 wraps), so every output word of round 1 is one
// table lookup on the varying word XORed with a constant of key and counter.
struct alignas(16) CtrConsts {
    uint32_t x0[3];   // BE32: counter words 0..2 after the initial AddRoundKey
    uint32_t kvar;    // initial round key word of the varying counter word (3 or 0)
    uint32_t p[4];    // round-1 constants, one per output word
};

struct HostTables {
    uint8_t sbox[256];
    uint8_t inv_sbox[256];
    uint32_t words[kTableWords];
};

// Builds the table image from the library's own GF(2^8) arithmetic.
const HostTables &host_tables();

// An expanded key with a consistent size and round count.
bool key_ok(const aesgpu_key *k);

// InvMixColumns of one little-endian column word (host).
uint32_t inv_mix_column(uint32_t w);

enum class Op { kEcbEnc, kEcbDec, kCtrBe32, kCtrLe128, kCbcDec };

struct LaunchArgs {
    Op op;
    uint32_t nr;
    const void *in;
    void *out;
    uint64_t n_bytes;     // ECB/CBC: 16 * n_blocks
    const RoundKeys *rk;  // enc keys for encryption/CTR, dec keys for decryption
    CtrConsts ctr;        // kCtrBe32, kCtrLe128
    uint32_t ctr0;        // kCtrBe32 only
    uint32_t iv[4];       // kCtrLe128 (counter of block 0), kCbcDec (IV words)
    uint64_t index0;      // kCtrLe128: added to iv (0 from the host's own calls)
    int bpl;              // blocks per lane: 1, 2 or 4, or 0 to choose by size
    uint32_t max_tiles;   // most tiles per CU in one kernel launch (a longer call is
                          // split), 0 = kMaxTilesPerCu
};

// A single-buffer kernel's workgroup hands out at most 16 * kMaxTilesPerCu
// shares of work from a 16-bit LDS count; longer calls are split into several
// launches.
constexpr uint32_t kMaxTilesPerCu = 4096;

// Enqueues the kernel for `a` on `stream`; returns an AESGPU status.
int launch(const uint32_t *d_tables, int n_cu, const LaunchArgs &a, hipStream_t stream);

// ---- small host helpers ------------------------------------------------------

inline uint32_t le32(const uint8_t *p) {
    return uint32_t(p[0]) | (uint32_t(p[1]) << 8) | (uint32_t(p[2]) << 16) | (uint32_t(p[3]) << 24);
}

// Makes `device` current for the lifetime of the guard.
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
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;
    bool ok() const { return ok_; }

  private:
    int prev_ = -1;
    bool ok_ = false;
};

}  // namespace aesgpu

struct aesgpu_ctx {
    int device;
    int n_cu;
    uint32_t *d_tables;
    int blocks_per_lane;   // single-buffer launches: 1, 2 or 4 (AESGPU_FORCE_BPL at
                           // create), 0 = chosen by size
    uint32_t max_tiles;    // single-buffer launches: tiles per CU per launch
                           // (AESGPU_MAX_TILES_PER_CU at create), 0 = kMaxTilesPerCu
};
