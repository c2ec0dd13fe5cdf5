// Continuous-batching AES server.
//
// Requests (encrypt or decrypt one device buffer in ECB with a key from a
// resident pool) enter a FIFO.  A dispatcher thread admits requests in order
// as long as their output fits in a device arena (best-fit ranges), and
// whenever one of its streams is idle it launches every admitted request as
// one batched run (the persistent kernel of the batched path, reading the
// pool's key schedules that stay resident on the device), or, for a batch of
// only a few requests, as one single-buffer launch per request.  Requests that
// arrive while earlier batches are still on the GPU are admitted and launched
// on the next free stream, so batches overlap on the device.  Completion is
// observed through one event per launch; outputs stay in the arena until the
// caller releases them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "aes_batch.h"
#include "aes_internal.h"

// ---- best-fit range allocator ----------------------------------------------------
//
// Free ranges are indexed twice: by offset (to coalesce on release) and by
// (size, offset) (to find the smallest range that fits in O(log n)).  A
// scan over the free list, as first fit does, costs O(free ranges) per
// allocation; the server admits thousands of requests in one batch under its
// lock, and a fragmented list then stalls the dispatcher.

struct aesgpu_arena {
    uint64_t capacity = 0;
    uint64_t granule = 256;
    uint64_t used = 0;
    uint64_t high_water = 0;
    std::map<uint64_t, uint64_t> free_ranges;           // offset -> length, non-adjacent
    std::set<std::pair<uint64_t, uint64_t>> by_size;    // (length, offset) of each free range
    std::map<uint64_t, uint64_t> live;                  // offset -> length of each allocation

    uint64_t round(uint64_t n) const { return (n + granule - 1) / granule * granule; }

    void add_free(uint64_t off, uint64_t len) {
        free_ranges.emplace(off, len);
        by_size.emplace(len, off);
    }
    void remove_free(std::map<uint64_t, uint64_t>::iterator it) {
        by_size.erase({it->second, it->first});
        free_ranges.erase(it);
    }

    // The smallest free range that fits (the lowest offset among equal
    // lengths); the allocation takes its start.
    bool alloc(uint64_t n, uint64_t *off) {
        const uint64_t need = round(n ? n : 1);
        auto fit = by_size.lower_bound({need, 0});
        if (fit == by_size.end()) return false;
        const uint64_t len = fit->first, at = fit->second;
        remove_free(free_ranges.find(at));
        if (len > need) add_free(at + need, len - need);
        live.emplace(at, need);
        used += need;
        high_water = std::max(high_water, used);
        *off = at;
        return true;
    }

    // Returns false unless [off, off + n) is exactly a live allocation.
    bool release(uint64_t off, uint64_t n) {
        const uint64_t len = round(n ? n : 1);
        auto a = live.find(off);
        if (a == live.end() || a->second != len) return false;
        live.erase(a);
        uint64_t start = off, size = len;
        auto next = free_ranges.lower_bound(off);
        if (next != free_ranges.end() && next->first == off + len) {
            size += next->second;
            auto after = std::next(next);
            remove_free(next);
            next = after;
        }
        if (next != free_ranges.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                size += prev->second;
                remove_free(prev);
            }
        }
        add_free(start, size);
        used -= len;
        return true;
    }

    uint64_t largest_free() const { return by_size.empty() ? 0 : by_size.rbegin()->first; }
};

extern "C" {

int aesgpu_arena_create(uint64_t capacity, uint64_t granule, aesgpu_arena **out) {
    if (!out) return AESGPU_EINVAL;
    *out = nullptr;
    if (!granule || (granule & (granule - 1)) || capacity % granule || !capacity)
        return AESGPU_EINVAL;
    aesgpu_arena *a = new (std::nothrow) aesgpu_arena;
    if (!a) return AESGPU_ENOMEM;
    a->capacity = capacity;
    a->granule = granule;
    a->add_free(0, capacity);
    *out = a;
    return AESGPU_OK;
}

int aesgpu_arena_alloc(aesgpu_arena *a, uint64_t n_bytes, uint64_t *offset) {
    if (!a || !offset) return AESGPU_EINVAL;
    if (a->round(n_bytes ? n_bytes : 1) > a->capacity) return AESGPU_EINVAL;
    return a->alloc(n_bytes, offset) ? AESGPU_OK : AESGPU_EAGAIN;
}

int aesgpu_arena_release(aesgpu_arena *a, uint64_t offset, uint64_t n_bytes) {
    if (!a) return AESGPU_EINVAL;
    return a->release(offset, n_bytes) ? AESGPU_OK : AESGPU_EINVAL;
}

int aesgpu_arena_query(const aesgpu_arena *a, uint64_t *used, uint64_t *largest_free,
                       uint64_t *high_water) {
    if (!a) return AESGPU_EINVAL;
    if (used) *used = a->used;
    if (largest_free) *largest_free = a->largest_free();
    if (high_water) *high_water = a->high_water;
    return AESGPU_OK;
}

void aesgpu_arena_destroy(aesgpu_arena *a) { delete a; }

}  // extern "C"

// ---- server ------------------------------------------------------------------------

using namespace aesgpu;

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    uint64_t id;
    uint32_t key;
    uint8_t dir;
    const void *in;
    uint64_t n;
    double t_arrival;
    uint64_t out_off;
    double t_launch;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *d_buf = nullptr;   // descriptors | tiles | counters
    size_t d_cap = 0;
    void *h_buf = nullptr;   // pinned staging of the same layout
    size_t h_cap = 0;
    uint32_t *d_counters = nullptr;  // the batch kernel's counters (kCounterBytes, kept zero)
    bool busy = false;
    std::vector<Req> reqs;
};

// Resident mode: a request's tiles and where they sit in their ring.
struct Pub {
    uint64_t first;   // ring index of the first tile
    uint64_t n;       // tiles
    bool done;
};

struct Live {
    Req req;
    uint32_t slot;    // tile counter and completion entry
    uint32_t set;     // ring
    uint64_t tile;    // blocks per tile
    uint64_t pub;     // publication number within the ring
};

}  // namespace

struct aesgpu_server {
    aesgpu_ctx *ctx = nullptr;
    aesgpu_server_config cfg{};
    size_t n_keys = 0;
    std::vector<uint16_t> key_bits;
    std::vector<uint32_t> h_sched;  // host copy of the schedules (direct launches)
    uint32_t *d_sched = nullptr;
    uint8_t *d_arena = nullptr;
    aesgpu_arena arena;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> waiting;
    std::deque<aesgpu_done> completed;
    std::vector<Slot> slots;
    std::thread worker;
    std::atomic<bool> stop{false};
    // Bumped by every submission and release (under mu); read without the
    // lock by the resident dispatcher to skip admission passes with nothing new.
    std::atomic<uint64_t> wake_gen{0};
    int fatal = AESGPU_OK;

    aesgpu_server_stats stats{};

    // Resident mode (AESGPU_SERVER_RESIDENT): one kernel stays on the GPU and
    // takes tiles from two rings in pinned host memory.
    bool resident = false;
    uint64_t ring_cap = 0;                      // entries per ring (power of two)
    ResTile *h_ring[2] = {nullptr, nullptr};    // host addresses
    ResTile *d_ring[2] = {nullptr, nullptr};    // device addresses
    uint64_t *h_ctl = nullptr, *d_ctl = nullptr;    // tails and stop word
    uint64_t *h_done = nullptr, *d_done = nullptr;  // completion ring (kResSlots entries)
    uint64_t done_head = 0;                     // completion entries consumed
    uint64_t *d_dev = nullptr;                  // the kernel's control block
    uint32_t *d_tiles_done = nullptr;           // per request slot
    hipStream_t res_stream = nullptr;
    hipEvent_t res_event = nullptr;
    bool res_running = false;
    bool res_restarting = false;                // stop requested to change the split
    double res_checked = 0;                     // last split check (server clock)
    uint64_t pending_blocks[2] = {0, 0};        // blocks of unfinished requests per ring
    uint32_t epoch = 0;
    uint32_t n_wg = 0, n_wg_forward = 0;
    uint64_t tail[2] = {0, 0};                  // published tiles per ring
    std::deque<Pub> pubs[2];                    // unfinished publications, oldest first
    uint64_t pub_base[2] = {0, 0};              // publication number of pubs[set].front()
    uint64_t pub_count[2] = {0, 0};
    std::vector<Live> live;                     // by slot: admitted, not yet complete
    size_t n_live = 0;
    std::vector<uint32_t> free_slots;
    std::vector<uint32_t> slot_tiles;           // tiles ever counted per slot (mod 2^32)

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

bool ensure(void **p, size_t *cap, size_t need, bool pinned) {
    if (*cap >= need) return true;
    size_t n = std::max(need, *cap * 2);
    if (*p) (void)(pinned ? hipHostFree(*p) : hipFree(*p));
    *p = nullptr;
    *cap = 0;
    const hipError_t e = pinned ? hipHostMalloc(p, n, hipHostMallocDefault) : hipMalloc(p, n);
    if (e != hipSuccess) {
        *p = nullptr;
        return false;
    }
    *cap = n;
    return true;
}

// Launches the requests in slot.reqs; returns an AESGPU status.  `backlog`:
// requests were still waiting after this batch was admitted.
int launch_slot(aesgpu_server *s, Slot &slot, bool backlog) {
    const size_t m = slot.reqs.size();
    if (!backlog && s->cfg.direct_requests != AESGPU_SERVER_NO_DIRECT &&
        m <= s->cfg.direct_requests) {
        // A few requests and none queued behind them: the single-buffer
        // kernel, round keys as kernel arguments.  Nothing is copied to the
        // device first, so a small batch costs its launches only, and each
        // request gets the whole chip.  Under a backlog the dispatcher thread
        // itself is the limit, and one batched launch per batch costs it less
        // than one launch per request.
        for (const Req &r : slot.reqs) {
            const bool dec = r.dir == AESGPU_DIR_DECRYPT;
            LaunchArgs a{};
            a.op = dec ? Op::kEcbDec : Op::kEcbEnc;
            a.nr = s->key_bits[r.key] / 32u + 6u;
            a.in = r.in;
            a.out = s->d_arena + r.out_off;
            a.n_bytes = r.n;
            a.rk = reinterpret_cast<const RoundKeys *>(
                s->h_sched.data() + size_t(r.key) * kSchedWords + (dec ? 64 : 0));
            a.bpl = s->ctx->blocks_per_lane;
            const int st = launch(s->ctx->d_tables, s->ctx->n_cu, a, slot.stream);
            if (st != AESGPU_OK) return st;
        }
        return hipEventRecord(slot.done, slot.stream) == hipSuccess ? AESGPU_OK : AESGPU_EHIP;
    }
    std::vector<aesgpu_msg> msgs(m);
    for (size_t i = 0; i < m; ++i) {
        const Req &r = slot.reqs[i];
        aesgpu_msg &x = msgs[i];
        std::memset(&x, 0, sizeof(x));
        x.in_off = reinterpret_cast<uintptr_t>(r.in);   // absolute input address
        x.out_off = r.out_off;                          // relative to the arena
        x.n_bytes = r.n;
        x.key_slot = r.key;
        x.key_bits = s->key_bits[r.key];
        x.mode = AESGPU_MODE_ECB;
        x.dir = r.dir;
    }
    uint32_t tile_blocks = s->cfg.tile_blocks;
    if (!tile_blocks) {
        // Adaptive: about two tiles per wave slot of this batch's share of
        // the CUs (the chip divided among it and the batches already in
        // flight), so that a small batch is still spread over many waves (a
        // lone wave on a long tile is latency bound) while batches of the
        // other streams keep CUs to run on; between one step and 8192 blocks.
        // The dispatcher thread alone sets and clears the busy flags.
        uint64_t blocks = 0;
        for (const Req &r : slot.reqs) blocks += r.n / 16;
        const uint64_t step = 64ull * s->cfg.blocks_per_lane;
        uint64_t running = 0;
        for (const Slot &o : s->slots) running += o.busy ? 1 : 0;
        const uint64_t share = std::max<uint64_t>(1, uint64_t(s->ctx->n_cu) / (1 + running));
        const uint64_t target = 2ull * share * 16;
        uint64_t tb = (blocks + target - 1) / target;
        tb = (tb + step - 1) / step * step;
        tile_blocks = uint32_t(std::min<uint64_t>(std::max<uint64_t>(tb, step), 8192));
    }
    std::vector<DevMsg> dm;
    std::vector<Tile> tiles[2];
    std::vector<uint32_t> cbc_list;   // stay empty: served requests are ECB
    std::vector<Tile> cbc_groups;
    BatchTotals tot;
    int st = build_tiles(msgs.data(), m, tile_blocks, dm, tiles, cbc_list, cbc_groups, tot);
    if (st != AESGPU_OK) return st;
    const size_t mb = m * sizeof(DevMsg), t0 = tiles[0].size() * sizeof(Tile),
                 t1 = tiles[1].size() * sizeof(Tile);
    const size_t bytes = mb + t0 + t1;
    if (!ensure(&slot.h_buf, &slot.h_cap, bytes, true) ||
        !ensure(&slot.d_buf, &slot.d_cap, bytes, false))
        return AESGPU_ENOMEM;
    char *h = static_cast<char *>(slot.h_buf);
    std::memcpy(h, dm.data(), mb);
    std::memcpy(h + mb, tiles[0].data(), t0);
    std::memcpy(h + mb + t0, tiles[1].data(), t1);
    if (hipMemcpyAsync(slot.d_buf, slot.h_buf, bytes, hipMemcpyHostToDevice, slot.stream) !=
        hipSuccess)
        return AESGPU_EHIP;
    const char *desc = static_cast<const char *>(slot.d_buf);
    BatchLaunch L{};
    L.msgs = reinterpret_cast<const DevMsg *>(desc);
    L.tiles[0] = reinterpret_cast<const Tile *>(desc + mb);
    L.tiles[1] = reinterpret_cast<const Tile *>(desc + mb + t0);
    L.n_tiles[0] = uint32_t(tiles[0].size());
    L.n_tiles[1] = uint32_t(tiles[1].size());
    L.counters = slot.d_counters;
    L.keys = nullptr;
    L.sched = s->d_sched;
    L.in = nullptr;
    L.out = s->d_arena;
    L.tables = s->ctx->d_tables;
    L.cbc_list = nullptr;
    L.cbc_groups = nullptr;
    L.cbc_dummy = nullptr;
    L.n_cbc_groups = 0;
    L.n_cu = s->ctx->n_cu;
    L.bpl = s->cfg.blocks_per_lane;
    L.blocks[0] = tot.blocks[0];
    L.blocks[1] = tot.blocks[1];
    st = enqueue_batch(L, slot.stream);
    if (st != AESGPU_OK) return st;
    return hipEventRecord(slot.done, slot.stream) == hipSuccess ? AESGPU_OK : AESGPU_EHIP;
}

void finish_slot(aesgpu_server *s, Slot &slot, int status, double t) {
    for (const Req &r : slot.reqs) {
        aesgpu_done d{};
        d.req_id = r.id;
        d.status = status;
        d.d_out = s->d_arena + r.out_off;
        d.n_bytes = r.n;
        d.t_arrival = r.t_arrival;
        d.t_launch = r.t_launch;
        d.t_done = t;
        s->completed.push_back(d);
        s->stats.requests_done++;
        s->stats.bytes_done += r.n;
    }
    slot.reqs.clear();
    slot.busy = false;
}

void worker_main(aesgpu_server *s) {
    if (hipSetDevice(s->ctx->device) != hipSuccess) {
        std::lock_guard<std::mutex> g(s->mu);
        s->fatal = AESGPU_EHIP;
        return;
    }
    uint64_t seen_gen = 0;  // wake_gen at the last admission attempt
    while (!s->stop.load(std::memory_order_acquire)) {
        bool in_flight = false;
        // 1. Completions.
        for (Slot &slot : s->slots) {
            if (!slot.busy) continue;
            const hipError_t q = hipEventQuery(slot.done);
            if (q == hipErrorNotReady) {
                in_flight = true;
                continue;
            }
            const double t = s->now();
            std::lock_guard<std::mutex> g(s->mu);
            finish_slot(s, slot, q == hipSuccess ? AESGPU_OK : AESGPU_EHIP, t);
        }
        // 2. Admission and launch on every idle stream.
        for (Slot &slot : s->slots) {
            if (slot.busy) continue;
            bool backlog = false;
            {
                std::lock_guard<std::mutex> g(s->mu);
                seen_gen = s->wake_gen.load(std::memory_order_relaxed);
                uint64_t bytes = 0;
                while (!s->waiting.empty()) {
                    Req &r = s->waiting.front();
                    if (s->cfg.max_batch_requests && slot.reqs.size() >= s->cfg.max_batch_requests)
                        break;
                    if (s->cfg.max_batch_bytes && !slot.reqs.empty() &&
                        bytes + r.n > s->cfg.max_batch_bytes)
                        break;
                    uint64_t off = 0;
                    if (!s->arena.alloc(r.n, &off)) break;  // FIFO: wait for memory
                    r.out_off = off;
                    bytes += r.n;
                    slot.reqs.push_back(r);
                    s->waiting.pop_front();
                }
                backlog = !s->waiting.empty();
            }
            if (slot.reqs.empty()) break;
            const double t = s->now();
            for (Req &r : slot.reqs) r.t_launch = t;
            const int st = launch_slot(s, slot, backlog);
            // A failed launch may have queued work that reads the staging
            // buffers or writes the arena: let it end before the requests
            // complete (and their outputs can be released and reused).
            if (st != AESGPU_OK) (void)hipStreamSynchronize(slot.stream);
            std::lock_guard<std::mutex> g(s->mu);
            s->stats.batches++;
            s->stats.max_batch_requests =
                std::max<uint64_t>(s->stats.max_batch_requests, slot.reqs.size());
            if (st != AESGPU_OK) {
                finish_slot(s, slot, st, s->now());
            } else {
                slot.busy = true;
                in_flight = true;
            }
        }
        // 3. Idle: sleep until a submission or a release (requests that wait
        // for arena memory need a release); busy: keep polling.
        if (!in_flight) {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait_for(lk, std::chrono::milliseconds(2), [&] {
                return s->stop.load() || s->wake_gen != seen_gen;
            });
        } else {
            std::this_thread::yield();
        }
    }
}

// ---- resident mode ---------------------------------------------------------------

constexpr uint64_t kResRing = uint64_t(1) << 16;   // tiles per ring
constexpr uint32_t kResSlots = 1u << 16;           // requests in flight at most
constexpr uint32_t kResIdlePolls = 25000;          // ≈ tens of ms without work, then the kernel ends

// Blocks per tile of a request in the resident kernel: spread it over the
// waves of its set that the requests already in flight leave free (a lone
// request gets them all), whole steps of the kernel, between 256 blocks
// and 8192, and never more tiles than half a ring.
uint64_t resident_tile_blocks(const aesgpu_server *s, uint32_t set, uint64_t n_blocks,
                              uint64_t live_in_set) {
    if (s->cfg.tile_blocks) return std::max<uint64_t>(s->cfg.tile_blocks,
                                                      (n_blocks + kResRing / 2 - 1) / (kResRing / 2));
    const uint64_t step = 64ull * s->cfg.blocks_per_lane;
    const uint64_t wgs = set ? s->n_wg - s->n_wg_forward : s->n_wg_forward;
    const uint64_t waves = std::max<uint64_t>(1, wgs * 16 - 1);
    const uint64_t share = std::max<uint64_t>(1, waves / (1 + live_in_set));
    uint64_t tb = (n_blocks + share - 1) / share;
    tb = (tb + step - 1) / step * step;
    tb = std::min<uint64_t>(std::max<uint64_t>(tb, std::max<uint64_t>(step, 256)), 8192);
    return std::max<uint64_t>(tb, (n_blocks + kResRing / 2 - 1) / (kResRing / 2));
}

// Workgroups for ring 0 (forward tables).  When the unfinished work is large
// (≥ kResSplitMin blocks, about a quarter millisecond of the chip) and its mix
// is at least an eighth of the chip away from the current split: in
// proportion to the blocks, between an eighth and seven eighths.  Otherwise
// the current split while the kernel runs, and half at a launch.
constexpr uint64_t kResSplitMin = uint64_t(1) << 24;
constexpr double kResSplitCheck = 2e-3;   // seconds between checks while running

uint32_t resident_split(const aesgpu_server *s, bool at_launch) {
    const uint64_t p0 = s->pending_blocks[0], p1 = s->pending_blocks[1];
    const uint32_t lo = std::max<uint32_t>(1, s->n_wg / 8), hi = s->n_wg - lo;
    if (p0 + p1 < kResSplitMin) return at_launch ? s->n_wg / 2 : s->n_wg_forward;
    const uint32_t want = uint32_t(std::min<double>(
        hi, std::max<double>(lo, double(s->n_wg) * double(p0) / double(p0 + p1) + 0.5)));
    const uint32_t cur = s->n_wg_forward;
    return (want > cur ? want - cur : cur - want) >= lo ? want : cur;
}

int launch_resident_kernel(aesgpu_server *s) {
    ResidentLaunch L{};
    L.ring[0] = s->d_ring[0];
    L.ring[1] = s->d_ring[1];
    L.ring_mask = s->ring_cap - 1;
    L.host_ctl = s->d_ctl;
    L.dev = s->d_dev;
    L.tiles_done = s->d_tiles_done;
    L.done_ring = s->d_done;
    L.done_mask = kResSlots - 1;
    L.sched = s->d_sched;
    L.tables = s->ctx->d_tables;
    L.n_wg = s->n_wg;
    L.n_wg_forward = s->n_wg_forward;
    L.bpl = s->cfg.blocks_per_lane;
    L.epoch = ++s->epoch;
    L.idle_polls = kResIdlePolls;
    int st = launch_resident(L, s->res_stream);
    if (st == AESGPU_OK && hipEventRecord(s->res_event, s->res_stream) != hipSuccess)
        st = AESGPU_EHIP;
    return st;
}

void worker_resident(aesgpu_server *s) {
    if (hipSetDevice(s->ctx->device) != hipSuccess) {
        std::lock_guard<std::mutex> g(s->mu);
        s->fatal = AESGPU_EHIP;
        return;
    }
    std::vector<Live> admitted;
    std::vector<aesgpu_done> finished;
    uint64_t seen_gen = 0;
    uint64_t live_in_set[2] = {0, 0};
    while (!s->stop.load(std::memory_order_acquire)) {
        // 1. Completions: the kernel appends a request's slot to the
        // completion ring once its last tile is stored; entry i carries the
        // tag i + 1, so an entry not yet written (or from the ring's previous
        // lap) is told apart.  At most kResSlots requests are in flight, so
        // the kernel never overtakes this reader.
        finished.clear();
        const double t = s->now();
        for (;;) {
            const uint64_t e = __atomic_load_n(&s->h_done[s->done_head & (kResSlots - 1)],
                                               __ATOMIC_ACQUIRE);
            if (uint32_t(e >> 32) != uint32_t(s->done_head + 1)) break;
            s->done_head++;
            Live &l = s->live[uint32_t(e)];
            aesgpu_done d{};
            d.req_id = l.req.id;
            d.status = AESGPU_OK;
            d.d_out = s->d_arena + l.req.out_off;
            d.n_bytes = l.req.n;
            d.t_arrival = l.req.t_arrival;
            d.t_launch = l.req.t_launch;
            d.t_done = t;
            finished.push_back(d);
            s->pubs[l.set][l.pub - s->pub_base[l.set]].done = true;
            s->free_slots.push_back(l.slot);
            live_in_set[l.set]--;
            s->pending_blocks[l.set] -= l.req.n / 16;
            s->n_live--;
        }
        for (int set = 0; set < 2; ++set) {
            while (!s->pubs[set].empty() && s->pubs[set].front().done) {
                s->pubs[set].pop_front();
                s->pub_base[set]++;
            }
        }
        // 2. Admission, in arrival order, while a request slot, ring space
        // and arena memory are free.  The lock is taken only when there are
        // completions to hand over, or a submission or release happened (a
        // pass that stopped for lack of a slot or ring space is retried after
        // completions, one that stopped for memory after a release): a loop
        // that takes it every time competes with the callers' submissions and
        // releases.
        admitted.clear();
        if (!finished.empty() || s->wake_gen.load(std::memory_order_acquire) != seen_gen) {
            std::lock_guard<std::mutex> g(s->mu);
            for (const aesgpu_done &d : finished) {
                s->completed.push_back(d);
                s->stats.requests_done++;
                s->stats.bytes_done += d.n_bytes;
            }
            seen_gen = s->wake_gen.load(std::memory_order_relaxed);
            uint64_t planned[2] = {0, 0};  // tiles of requests admitted in this pass
            while (!s->waiting.empty() && !s->free_slots.empty()) {
                Req &r = s->waiting.front();
                const uint32_t set = r.dir == AESGPU_DIR_DECRYPT ? 1u : 0u;
                const uint64_t nb = r.n / 16;
                const uint64_t tb =
                    resident_tile_blocks(s, set, nb, live_in_set[set] + admitted.size());
                const uint64_t k = (nb + tb - 1) / tb;
                const uint64_t head = s->pubs[set].empty() ? s->tail[set] : s->pubs[set].front().first;
                if (s->tail[set] + planned[set] + k - head > s->ring_cap) break;
                uint64_t off = 0;
                if (!s->arena.alloc(r.n, &off)) break;  // FIFO: wait for memory
                r.out_off = off;
                Live l{};
                l.req = r;
                l.slot = s->free_slots.back();
                s->free_slots.pop_back();
                l.set = set;
                l.tile = tb;
                admitted.push_back(l);
                planned[set] += k;
                s->waiting.pop_front();
            }
            if (!admitted.empty()) {
                s->stats.max_batch_requests =
                    std::max<uint64_t>(s->stats.max_batch_requests, admitted.size());
            }
        }
        // 3. Publication: tile records first, then the tails.
        if (!admitted.empty()) {
            const double tl = s->now();
            for (Live &l : admitted) {
                const uint64_t tb = l.tile, nb = l.req.n / 16, k = (nb + tb - 1) / tb;
                const uint32_t nr = s->key_bits[l.req.key] / 32u + 6u;
                const uint64_t in = reinterpret_cast<uintptr_t>(l.req.in);
                const uint64_t out = reinterpret_cast<uintptr_t>(s->d_arena + l.req.out_off);
                for (uint64_t i = 0; i < k; ++i) {
                    ResTile &r = s->h_ring[l.set][(s->tail[l.set] + i) & (s->ring_cap - 1)];
                    r.in = in + 16 * i * tb;
                    r.out = out + 16 * i * tb;
                    r.n_blocks = uint32_t(std::min<uint64_t>(tb, nb - i * tb));
                    r.key_slot = l.req.key;
                    r.nr = nr;
                    r.req_slot = l.slot;
                    r.target = s->slot_tiles[l.slot] + uint32_t(k);
                }
                s->slot_tiles[l.slot] += uint32_t(k);
                s->pubs[l.set].push_back(Pub{s->tail[l.set], k, false});
                l.pub = s->pub_count[l.set]++;
                s->tail[l.set] += k;
                l.req.t_launch = tl;
                live_in_set[l.set]++;
                s->pending_blocks[l.set] += nb;
                s->live[l.slot] = l;
                s->n_live++;
            }
            std::atomic_thread_fence(std::memory_order_release);
            __atomic_store_n(&s->h_ctl[0], s->tail[0], __ATOMIC_RELEASE);
            __atomic_store_n(&s->h_ctl[1], s->tail[1], __ATOMIC_RELEASE);
        }
        // 4. The kernel: relaunched whenever requests are unfinished and it
        // has ended (it ends after a while without new tiles).  While it
        // runs, a backlog whose direction mix is far from the workgroups'
        // split stops it, and the next launch splits them anew.
        if (s->res_running) {
            const hipError_t q = hipEventQuery(s->res_event);
            if (q != hipErrorNotReady) {
                s->res_running = false;
                if (s->res_restarting) {
                    __atomic_store_n(&s->h_ctl[2], uint64_t(0), __ATOMIC_RELEASE);
                    s->res_restarting = false;
                }
                if (q != hipSuccess) {
                    std::lock_guard<std::mutex> g(s->mu);
                    s->fatal = AESGPU_EHIP;
                }
            } else if (!s->res_restarting && t - s->res_checked > kResSplitCheck) {
                s->res_checked = t;
                if (resident_split(s, false) != s->n_wg_forward) {
                    __atomic_store_n(&s->h_ctl[2], uint64_t(1), __ATOMIC_RELEASE);
                    s->res_restarting = true;
                    std::lock_guard<std::mutex> g(s->mu);
                    s->stats.rebalances++;
                }
            }
        }
        if (!s->res_running && s->n_live) {
            s->n_wg_forward = resident_split(s, true);
            const int st = launch_resident_kernel(s);
            std::lock_guard<std::mutex> g(s->mu);
            if (st != AESGPU_OK) {
                // Nothing will complete the requests in flight: fail them.
                s->fatal = st;
                const double tf = s->now();
                std::vector<bool> is_free(kResSlots, false);
                for (uint32_t f : s->free_slots) is_free[f] = true;
                for (uint32_t slot = 0; slot < kResSlots; ++slot) {
                    if (is_free[slot]) continue;
                    const Live &l = s->live[slot];
                    aesgpu_done d{};
                    d.req_id = l.req.id;
                    d.status = st;
                    d.d_out = s->d_arena + l.req.out_off;
                    d.n_bytes = l.req.n;
                    d.t_arrival = l.req.t_arrival;
                    d.t_launch = l.req.t_launch;
                    d.t_done = tf;
                    s->completed.push_back(d);
                    s->stats.requests_done++;
                }
                s->n_live = 0;
                return;
            }
            s->res_running = true;
            s->stats.batches++;
        }
        // 5. Idle: sleep until a submission or a release; busy: keep polling.
        if (!s->n_live) {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait_for(lk, std::chrono::milliseconds(2), [&] {
                return s->stop.load() || s->wake_gen != seen_gen;
            });
        } else {
            std::this_thread::yield();
        }
    }
}

void destroy_server(aesgpu_server *s) {
    if (s->worker.joinable()) {
        s->stop.store(true, std::memory_order_release);
        s->cv.notify_all();
        s->worker.join();
    }
    DeviceGuard g(s->ctx->device);
    if (s->res_stream) {
        // Ask the resident kernel to end and wait for it (it also ends by
        // itself after a while without work).
        if (s->h_ctl) __atomic_store_n(&s->h_ctl[2], uint64_t(1), __ATOMIC_RELEASE);
        (void)hipStreamSynchronize(s->res_stream);
        if (s->res_event) (void)hipEventDestroy(s->res_event);
        (void)hipStreamDestroy(s->res_stream);
    }
    for (void *h : {static_cast<void *>(s->h_ring[0]), static_cast<void *>(s->h_ring[1]),
                    static_cast<void *>(s->h_ctl), static_cast<void *>(s->h_done)})
        if (h) (void)hipHostFree(h);
    if (s->d_dev) (void)hipFree(s->d_dev);
    if (s->d_tiles_done) (void)hipFree(s->d_tiles_done);
    for (Slot &slot : s->slots) {
        if (slot.stream) (void)hipStreamSynchronize(slot.stream);
        if (slot.done) (void)hipEventDestroy(slot.done);
        if (slot.stream) (void)hipStreamDestroy(slot.stream);
        if (slot.d_buf) (void)hipFree(slot.d_buf);
        if (slot.d_counters) (void)hipFree(slot.d_counters);
        if (slot.h_buf) (void)hipHostFree(slot.h_buf);
    }
    if (s->d_sched) (void)hipFree(s->d_sched);
    if (s->d_arena) (void)hipFree(s->d_arena);
    delete s;
}

}  // namespace

extern "C" {

int aesgpu_server_create(aesgpu_ctx *ctx, const uint8_t *keys, const uint16_t *key_bits,
                         size_t n_keys, const aesgpu_server_config *cfg, aesgpu_server **out) {
    if (!out) return AESGPU_EINVAL;
    *out = nullptr;
    if (!ctx || !keys || !key_bits || n_keys == 0 || !cfg) return AESGPU_EINVAL;
    aesgpu_server_config c = *cfg;
    if (!c.n_streams) c.n_streams = 4;
    if (!c.blocks_per_lane) c.blocks_per_lane = 2;
    if (!c.max_queued) c.max_queued = 1u << 20;
    if (!c.direct_requests) c.direct_requests = 4;
    if ((c.flags & ~uint32_t(AESGPU_SERVER_RESIDENT)) || c.n_streams > 8 ||
        (c.blocks_per_lane != 1 && c.blocks_per_lane != 2 && c.blocks_per_lane != 4) ||
        c.tile_blocks % (64u * c.blocks_per_lane) || c.arena_bytes < 256 || c.arena_bytes % 256 ||
        (c.direct_requests > 16 && c.direct_requests != AESGPU_SERVER_NO_DIRECT))
        return AESGPU_EINVAL;
    // Expand every pool key on the host (encryption and decryption schedules).
    std::vector<uint32_t> sched(n_keys * kSchedWords, 0u);
    for (size_t i = 0; i < n_keys; ++i) {
        aesgpu_key k;
        const int st = aesgpu_expand_key(keys + 32 * i, key_bits[i] / 8, &k);
        if (st != AESGPU_OK) return st;
        std::memcpy(&sched[i * kSchedWords], k.enc, sizeof(k.enc));
        std::memcpy(&sched[i * kSchedWords + 64], k.dec, sizeof(k.dec));
    }
    aesgpu_server *s = new (std::nothrow) aesgpu_server;
    if (!s) return AESGPU_ENOMEM;
    s->ctx = ctx;
    s->cfg = c;
    s->n_keys = n_keys;
    s->key_bits.assign(key_bits, key_bits + n_keys);
    s->h_sched = sched;
    s->arena.capacity = c.arena_bytes;
    s->arena.granule = 256;
    s->arena.add_free(0, c.arena_bytes);
    // Resident mode runs on one stream of its own: no batch slots.
    s->slots.resize((c.flags & AESGPU_SERVER_RESIDENT) ? 0 : c.n_streams);
    s->t0 = Clock::now();
    {
        DeviceGuard g(ctx->device);
        bool ok = g.ok();
        ok = ok && hipMalloc(&s->d_sched, sched.size() * 4) == hipSuccess;
        ok = ok && hipMemcpy(s->d_sched, sched.data(), sched.size() * 4, hipMemcpyHostToDevice) ==
                       hipSuccess;
        ok = ok && hipMalloc(&s->d_arena, c.arena_bytes) == hipSuccess;
        const std::vector<uint8_t> zeros(kCounterBytes, 0);
        for (Slot &slot : s->slots) {
            ok = ok && hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&slot.done, hipEventDisableTiming) == hipSuccess;
            ok = ok && hipMalloc(&slot.d_counters, kCounterBytes) == hipSuccess;
            ok = ok && hipMemcpy(slot.d_counters, zeros.data(), kCounterBytes,
                                 hipMemcpyHostToDevice) == hipSuccess;
        }
        if (ok && (c.flags & AESGPU_SERVER_RESIDENT)) {
            s->resident = true;
            s->ring_cap = kResRing;
            s->n_wg = uint32_t(std::min(std::max(ctx->n_cu, 2), 1024));
            s->n_wg_forward = s->n_wg / 2;
            // Fine-grained (coherent) pinned memory: the kernel polls it while
            // the host writes it, and the reverse.
            const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
            auto mapped = [&](size_t n, void **h, void **d) {
                return hipHostMalloc(h, n, fl) == hipSuccess && *h &&
                       hipHostGetDevicePointer(d, *h, 0) == hipSuccess && *d;
            };
            void *h = nullptr, *d = nullptr;
            for (int set = 0; set < 2 && ok; ++set) {
                h = d = nullptr;
                ok = mapped(kResRing * sizeof(ResTile), &h, &d);
                s->h_ring[set] = static_cast<ResTile *>(h);
                s->d_ring[set] = static_cast<ResTile *>(d);
            }
            h = d = nullptr;
            ok = ok && mapped(64, &h, &d);
            s->h_ctl = static_cast<uint64_t *>(h);
            s->d_ctl = static_cast<uint64_t *>(d);
            h = d = nullptr;
            ok = ok && mapped(size_t(kResSlots) * 8, &h, &d);
            s->h_done = static_cast<uint64_t *>(h);
            s->d_done = static_cast<uint64_t *>(d);
            if (ok) {
                std::memset(s->h_ctl, 0, 64);
                std::memset(s->h_done, 0, size_t(kResSlots) * 8);
            }
            const size_t dev_bytes = res_dev_words(s->n_wg) * 8;
            const std::vector<uint8_t> zeros(std::max(dev_bytes, size_t(kResSlots) * 4), 0);
            ok = ok && hipMalloc(&s->d_dev, dev_bytes) == hipSuccess &&
                 hipMemcpy(s->d_dev, zeros.data(), dev_bytes, hipMemcpyHostToDevice) == hipSuccess;
            ok = ok && hipMalloc(&s->d_tiles_done, size_t(kResSlots) * 4) == hipSuccess &&
                 hipMemcpy(s->d_tiles_done, zeros.data(), size_t(kResSlots) * 4,
                           hipMemcpyHostToDevice) == hipSuccess;
            ok = ok && hipStreamCreateWithFlags(&s->res_stream, hipStreamNonBlocking) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&s->res_event, hipEventDisableTiming) == hipSuccess;
            if (ok) {
                s->slot_tiles.assign(kResSlots, 0u);
                s->live.resize(kResSlots);
                s->free_slots.reserve(kResSlots);
                for (uint32_t i = kResSlots; i > 0; --i) s->free_slots.push_back(i - 1);
            }
        }
        if (!ok) {
            destroy_server(s);
            return AESGPU_EHIP;
        }
    }
    try {
        s->worker = std::thread(s->resident ? worker_resident : worker_main, s);
    } catch (...) {
        destroy_server(s);
        return AESGPU_ENOMEM;
    }
    *out = s;
    return AESGPU_OK;
}

double aesgpu_server_now(const aesgpu_server *s) { return s ? s->now() : 0.0; }

}  // extern "C"

namespace {

int check_request(const aesgpu_server *s, int dir, uint32_t key_id, const void *d_in,
                  size_t n_bytes) {
    if (dir != AESGPU_DIR_ENCRYPT && dir != AESGPU_DIR_DECRYPT) return AESGPU_EINVAL;
    if (key_id >= s->n_keys) return AESGPU_EINVAL;
    if (n_bytes % 16 || uint64_t(n_bytes) > s->cfg.arena_bytes) return AESGPU_EINVAL;
    if (n_bytes && !d_in) return AESGPU_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_in) & 15u) return AESGPU_EALIGN;
    return AESGPU_OK;
}

// Queues one checked request; the caller holds s->mu and wakes the
// dispatcher afterwards.
int enqueue_locked(aesgpu_server *s, uint64_t req_id, int dir, uint32_t key_id,
                   const void *d_in, size_t n_bytes, double t_arrival) {
    if (s->fatal != AESGPU_OK) return s->fatal;
    if (n_bytes == 0) {
        aesgpu_done d{};
        d.req_id = req_id;
        d.t_arrival = t_arrival;
        d.t_launch = d.t_done = s->now();
        s->completed.push_back(d);
        return AESGPU_OK;
    }
    if (s->waiting.size() >= s->cfg.max_queued) return AESGPU_EAGAIN;
    s->waiting.push_back(Req{req_id, key_id, uint8_t(dir), d_in, n_bytes, t_arrival, 0, 0.0});
    s->stats.requests_submitted++;
    return AESGPU_OK;
}

}  // namespace

extern "C" {

int aesgpu_server_submit(aesgpu_server *s, uint64_t req_id, int dir, uint32_t key_id,
                         const void *d_in, size_t n_bytes, double t_arrival) {
    if (!s) return AESGPU_EINVAL;
    const int c = check_request(s, dir, key_id, d_in, n_bytes);
    if (c != AESGPU_OK) return c;
    std::lock_guard<std::mutex> g(s->mu);
    const int st = enqueue_locked(s, req_id, dir, key_id, d_in, n_bytes, t_arrival);
    if (st == AESGPU_OK) {
        s->wake_gen.fetch_add(1, std::memory_order_release);
        s->cv.notify_one();
    }
    return st;
}

int aesgpu_server_poll(aesgpu_server *s, aesgpu_done *out, size_t cap, size_t *n_out) {
    if (!s || !n_out || (cap && !out)) return AESGPU_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    size_t n = 0;
    while (n < cap && !s->completed.empty()) {
        out[n++] = s->completed.front();
        s->completed.pop_front();
    }
    *n_out = n;
    return AESGPU_OK;
}

int aesgpu_server_release(aesgpu_server *s, const void *d_out, size_t n_bytes) {
    if (!s) return AESGPU_EINVAL;
    if (n_bytes == 0) return AESGPU_OK;
    const uintptr_t p = reinterpret_cast<uintptr_t>(d_out), b = reinterpret_cast<uintptr_t>(s->d_arena);
    if (p < b || p - b >= s->cfg.arena_bytes) return AESGPU_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->arena.release(p - b, n_bytes)) return AESGPU_EINVAL;
    s->wake_gen.fetch_add(1, std::memory_order_release);
    s->cv.notify_one();
    return AESGPU_OK;
}

int aesgpu_server_get_stats(aesgpu_server *s, aesgpu_server_stats *out) {
    if (!s || !out) return AESGPU_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->queued = s->waiting.size();
    out->arena_used = s->arena.used;
    out->arena_high_water = s->arena.high_water;
    return AESGPU_OK;
}

int aesgpu_server_replay(aesgpu_server *s, const aesgpu_request *reqs, size_t n, double t_start,
                         aesgpu_done *done) {
    if (!s || (n && (!reqs || !done))) return AESGPU_EINVAL;
    std::vector<uint8_t> seen(n, 0);
    size_t n_done = 0, next = 0;
    std::vector<aesgpu_done> buf(256);
    while (n_done < n) {
        // Submit everything whose arrival time has come, under one lock.
        const double t_now = s->now();
        size_t end = next;
        while (end < n && t_now >= t_start + reqs[end].t_arrival) {
            const aesgpu_request &r = reqs[end];
            if (r.req_id >= n) return AESGPU_EINVAL;
            const int c = check_request(s, int(r.dir), r.key_id, r.d_in, r.n_bytes);
            if (c != AESGPU_OK) return c;
            ++end;
        }
        if (end > next) {
            std::lock_guard<std::mutex> g(s->mu);
            const size_t first = next;
            for (; next < end; ++next) {
                const aesgpu_request &r = reqs[next];
                const int st = enqueue_locked(s, r.req_id, int(r.dir), r.key_id, r.d_in,
                                              r.n_bytes, t_start + r.t_arrival);
                if (st == AESGPU_EAGAIN) break;
                if (st != AESGPU_OK) return st;
            }
            if (next > first) {
                s->wake_gen.fetch_add(1, std::memory_order_release);
                s->cv.notify_one();
            }
        }
        size_t got = 0;
        aesgpu_server_poll(s, buf.data(), buf.size(), &got);
        int status = AESGPU_OK;
        for (size_t i = 0; i < got; ++i) {
            const aesgpu_done &d = buf[i];
            if (d.req_id >= n || seen[d.req_id]) return AESGPU_EINVAL;
            seen[d.req_id] = 1;
            done[d.req_id] = d;
            ++n_done;
            if (d.status != AESGPU_OK && status == AESGPU_OK) status = d.status;
        }
        if (got) {
            // The polled outputs go back to the arena under one lock.
            std::lock_guard<std::mutex> g(s->mu);
            const uintptr_t b = reinterpret_cast<uintptr_t>(s->d_arena);
            for (size_t i = 0; i < got; ++i)
                if (buf[i].n_bytes)
                    (void)s->arena.release(reinterpret_cast<uintptr_t>(buf[i].d_out) - b,
                                           buf[i].n_bytes);
            s->wake_gen.fetch_add(1, std::memory_order_release);
            s->cv.notify_one();
        }
        if (status != AESGPU_OK) return status;
        if (!got) std::this_thread::yield();
    }
    return AESGPU_OK;
}

void aesgpu_server_destroy(aesgpu_server *s) {
    if (s) destroy_server(s);
}

}  // extern "C"
