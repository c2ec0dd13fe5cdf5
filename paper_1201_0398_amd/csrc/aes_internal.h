// Internal declarations shared by the host runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

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
};

// Enqueues the kernel for `a` on `stream`; returns an AESGPU status.
int launch(const uint32_t *d_tables, int n_cu, const LaunchArgs &a, hipStream_t stream);

// ---- batched launches --------------------------------------------------------

// Device descriptor of one message (64 bytes).
struct alignas(16) DevMsg {
    uint64_t in_off;
    uint64_t out_off;
    uint64_t n_full;    // whole blocks
    uint32_t tail;      // bytes of a final partial block (CTR only)
    uint32_t key_slot;
    uint32_t nr;
    uint32_t mode;      // AESGPU_MODE_ECB / CTR / CBC
    uint32_t nonce[3];  // CTR nonce words; CBC: IV words 0..2
    uint32_t ctr0;      // CTR first counter; CBC: IV word 3
    uint32_t pad[2];
};
static_assert(sizeof(DevMsg) == 64, "descriptor layout");

// A message-pure run of blocks (16 bytes), or a CBC-encryption group.
struct alignas(16) Tile {
    uint32_t msg;
    uint32_t n_blocks;      // blocks in this tile (the partial CTR block counts)
    uint64_t first_block;   // first block of the tile within its message
};
static_assert(sizeof(Tile) == 16, "tile layout");

// A CBC-encryption group (same 16-byte layout): up to 64 CBC-encrypt messages
// of one key size, one lane each (encryption is sequential within a message);
// msg is the group's first index into the CBC list, n_blocks its message
// count, first_block its longest message's block count.

// Words per key slot of a resident schedule: 64 encryption words (60 used)
// followed by 64 equivalent-inverse-cipher words.
constexpr uint32_t kSchedWords = 128;

// Device bytes after the tiles: 2 queue counters (zero before each run) and
// one scratch flag per workgroup (at most 1024 workgroups).
constexpr size_t kCounterBytes = 4 * (2 + 1024) + 56;

struct BatchTotals {
    uint64_t total = 0;    // sum of message bytes
    uint64_t blocks[2] = {0, 0};  // blocks per table set
    uint64_t in_end = 0;   // max(in_off + n_bytes)
    uint64_t out_end = 0;  // max(out_off + n_bytes)
    uint32_t max_slot = 0;
    bool cbc_dec_self_overlap = false;  // a CBC-decrypt message whose input and output ranges meet
};

// Everything one batched run needs on the device.  Set 0 is the forward
// table set (ECB encryption, CTR), set 1 the inverse set (ECB decryption).
// Both sets run in one launch.
struct BatchLaunch {
    const DevMsg *msgs;
    const Tile *tiles[2];
    uint32_t n_tiles[2];
    uint32_t *counters;      // kCounterBytes: two tile counters, then per-workgroup flags
    const uint8_t *keys;     // raw keys (expanded on the device), or
    const uint32_t *sched;   // resident schedules (kSchedWords per slot)
    const uint8_t *in;
    uint8_t *out;
    const uint32_t *tables;
    const uint32_t *cbc_list;  // message indices of the CBC-encryption groups
    const Tile *cbc_groups;    // the groups, longest first (own launch)
    uint4 *cbc_dummy;          // 16 scratch bytes for stores with nothing to store
    uint32_t n_cbc_groups;
    int n_cu;
    uint32_t bpl;
    uint64_t blocks[2];      // blocks per set, to split the workgroups
    bool reset_counters;     // launch a counter reset first (else already zero)
};

// Validates messages and cuts them into tiles of at most tile_blocks blocks,
// each queue sorted longest first; CBC-encrypt messages form groups (per key
// size, longest first, listed in cbc_list) for their own launch.
int build_tiles(const aesgpu_msg *msgs, size_t m, uint32_t tile_blocks, std::vector<DevMsg> &dm,
                std::vector<Tile> (&tiles)[2], std::vector<uint32_t> &cbc_list,
                std::vector<Tile> &cbc_groups, BatchTotals &tot);

// Optional counter reset, then one persistent launch over both queues, then
// (if the batch has CBC-encrypt messages) the CBC-encryption launch.
int enqueue_batch(const BatchLaunch &L, hipStream_t stream);

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
};
