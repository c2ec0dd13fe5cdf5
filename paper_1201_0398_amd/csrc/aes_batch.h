// Internal declarations of the batched launches (planner, persistent
// launch, CBC-encryption launch), shared by the batch and server sources.
#pragma once

#include <vector>

#include "aes_internal.h"

namespace aesgpu {

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

// A CBC-encryption group (same 16-byte layout): up to kCbcGroupMsgs
// CBC-encrypt messages of one key size, four lanes each (encryption is
// sequential within a message); msg is the group's first index into the CBC
// list, n_blocks its message count, first_block its longest message's block
// count.
constexpr uint32_t kCbcGroupMsgs = 16;

// Words per key slot of a resident schedule: 64 encryption words (60 used)
// followed by 64 equivalent-inverse-cipher words.
constexpr uint32_t kSchedWords = 128;

// Device bytes of a launch's counters: 2 queue counters, one scratch flag per
// workgroup (at most 1024 workgroups), then the count of workgroups that have
// finished.  The counters must be zero before the first launch; the last
// workgroup of every launch zeroes the queue counters and the count again.
constexpr size_t kCounterBytes = 4 * (2 + 1024) + 56;
constexpr uint32_t kExitWord = 2 + 1024;

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
    uint32_t *counters;      // kCounterBytes, zero before the launch (see kCounterBytes)
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
};

// Validates messages and cuts them into tiles of at most tile_blocks blocks,
// each queue sorted longest first; CBC-encrypt messages form groups (per key
// size, longest first, listed in cbc_list) for their own launch.
int build_tiles(const aesgpu_msg *msgs, size_t m, uint32_t tile_blocks, std::vector<DevMsg> &dm,
                std::vector<Tile> (&tiles)[2], std::vector<uint32_t> &cbc_list,
                std::vector<Tile> &cbc_groups, BatchTotals &tot);

// One persistent launch over both queues, then (if the batch has CBC-encrypt
// messages) the CBC-encryption launch.
int enqueue_batch(const BatchLaunch &L, hipStream_t stream);

// ---- resident serving kernel ----------------------------------------------------
//
// One ECB tile of a served request, written by the host into a ring in
// pinned host memory and read by the kernel over the host link.
struct alignas(64) ResTile {
    uint64_t in;        // device address of the tile's first input block
    uint64_t out;       // device address of its first output block
    uint32_t n_blocks;  // blocks in this tile
    uint32_t key_slot;
    uint32_t nr;
    uint32_t req_slot;  // the request's slot (tile counter, completion entry)
    uint32_t target;    // the slot's tile count (mod 2^32) once the request is done
    uint32_t pad[7];
};
static_assert(sizeof(ResTile) == 64, "resident tile layout");

// Host control words (pinned, written by the host): published tail of each
// ring (tiles 0 .. tail - 1 are valid), then the stop request.
constexpr uint32_t kResHostWords = 3;

// Device control block, in 64-bit words, each group on a 128-byte line of its
// own: the ticket counter of each set at word 16 * set, the count of finished
// requests at word 32 and the count of waves that have ended at word 40, and
// from word 48 + 16 * w workgroup w's copies of the tails of ring 0 and ring 1
// and its stop word (the launch epoch that must stop).  Zero before the first
// launch.
constexpr size_t kResDoneWord = 32;
constexpr size_t kResExitWord = 40;
constexpr size_t kResCopyWord = 48;
constexpr size_t res_dev_words(uint32_t n_wg) { return kResCopyWord + 16 * size_t(n_wg); }

struct ResidentLaunch {
    const ResTile *ring[2];     // device addresses of the two host rings
    uint64_t ring_mask;         // ring entries - 1 (a power of two)
    const uint64_t *host_ctl;   // device address of the host control words
    uint64_t *dev;              // device control block
    uint32_t *tiles_done;       // per request slot: tiles finished, only grows (mod 2^32)
    uint64_t *done_ring;        // device address of the host completion ring: entry
                                // i % (done_mask + 1) = (i + 1) << 32 | slot, written
                                // once the i-th request (in finishing order) is done
    uint64_t done_mask;
    const uint32_t *sched;      // resident schedules (kSchedWords per key slot)
    const uint32_t *tables;
    uint32_t n_wg;              // workgroups (one per CU at most)
    uint32_t n_wg_forward;      // the first n_wg_forward serve ring 0 (forward tables);
                                // may change from one launch to the next
    uint32_t bpl;
    uint32_t epoch;             // launch number, distinguishes stop requests
    uint32_t idle_polls;        // polls without work before the kernel ends
};

// Launches the resident kernel; it ends when the host sets the stop word or
// after idle_polls polls without new work.
int launch_resident(const ResidentLaunch &L, hipStream_t stream);

}  // namespace aesgpu
