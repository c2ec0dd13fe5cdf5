// Host-staged pipeline: host buffers in, host buffers out.
//
// The paper's section 3 moves every buffer across the bus: the input is
// mapped into a texture, drawn, and the output read back, and its section 3.1
// finds the GPU slower than the CPU for small data because of that transfer
// cost.  This is the same data path done as a pipeline: the buffer is cut
// into chunks that run on several streams, so the transfers of one chunk
// overlap the device work of the others.  Host buffers allocated with
// aesgpu_host_alloc() (pinned and mapped into the device's address space)
// need no staging: by default the kernel reads its input from and writes its
// output to host memory directly over PCIe (zero copy), so both directions of
// the link are busy at once.  Pageable host memory goes through pinned,
// mapped staging buffers: a CPU copy, split over a few threads, fills a
// chunk's input staging buffer, the kernel reads it and writes the output
// staging buffer over the link, and a CPU copy moves that to the caller while
// the other slots' kernels run.  With AESGPU_PIPELINE_COPY each chunk is
// instead moved to device buffers and back by DMA copies on its stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "aes_internal.h"

using namespace aesgpu;

namespace {

constexpr size_t kDefaultChunk = size_t(8) << 20;
constexpr int kDefaultSlots = 3;
constexpr int kMaxSlots = 16;

struct Pinned {
    size_t size;
    uintptr_t device;   // the allocation's address in the device's address space
};

// Pinned allocations made by aesgpu_host_alloc(): host base -> allocation.
std::mutex g_pinned_mu;
std::map<uintptr_t, Pinned> g_pinned;

// Device address of [p, p + n) when it lies inside one aesgpu_host_alloc()
// allocation, else 0.
uintptr_t pinned_device_address(const void *p, size_t n) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(p);
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    auto it = g_pinned.upper_bound(x);
    if (it == g_pinned.begin()) return 0;
    --it;
    const uintptr_t d = x - it->first;
    if (d > it->second.size || n > it->second.size - d) return 0;
    return it->second.device + d;
}

bool ranges_overlap(const void *a, const void *b, size_t n) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y ? y - x < n : x - y < n;
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *d_in = nullptr, *d_out = nullptr;   // device chunk buffers (DMA copies)
    void *h_in = nullptr, *h_out = nullptr;   // pinned staging
    void *hd_in = nullptr, *hd_out = nullptr; // the staging buffers' device addresses
    bool busy = false;
    uint64_t off = 0, len = 0;                // chunk in flight
    bool staged_out = false;
};

// Host copies split over a few threads: one thread's memcpy reaches only a
// part of the host's memory bandwidth, and the staging copies bound the
// pageable path.  The calling thread copies one part itself.  Not
// reentrant: one copy at a time.
class CopyPool {
  public:
    static constexpr int kThreads = 4;            // including the caller
    static constexpr size_t kMinSplit = 1u << 20;  // smaller copies stay on one thread

    CopyPool() {
        try {
            for (int i = 1; i < kThreads; ++i) workers_.emplace_back([this, i] { work(i); });
        } catch (...) {
            shutdown();  // no threads: every copy runs on the caller
        }
    }
    ~CopyPool() { shutdown(); }

    void copy(void *dst, const void *src, size_t n) {
        if (n < kMinSplit || workers_.empty()) {
            std::memcpy(dst, src, n);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            dst_ = static_cast<char *>(dst);
            src_ = static_cast<const char *>(src);
            n_ = n;
            pending_ = int(workers_.size());
            ++gen_;
        }
        cv_.notify_all();
        part(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return pending_ == 0; });
    }

  private:
    void shutdown() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (std::thread &t : workers_) t.join();
        workers_.clear();
    }

    // Part i of the current copy: kThreads pieces, cut at 4 KiB multiples.
    void part(int i) {
        const size_t piece = (n_ / kThreads + 4095) & ~size_t(4095);
        const size_t a = std::min(n_, piece * size_t(i));
        const size_t b = i == kThreads - 1 ? n_ : std::min(n_, a + piece);
        if (b > a) std::memcpy(dst_ + a, src_ + a, b - a);
    }

    void work(int i) {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            part(i);
            std::lock_guard<std::mutex> lk(mu_);
            if (--pending_ == 0) done_cv_.notify_one();
        }
    }

    std::vector<std::thread> workers_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    uint64_t gen_ = 0;
    int pending_ = 0;
    bool stop_ = false;
    char *dst_ = nullptr;
    const char *src_ = nullptr;
    size_t n_ = 0;
};

}  // namespace

struct aesgpu_pipeline {
    aesgpu_ctx *ctx = nullptr;
    int device = 0;
    size_t chunk = 0;
    uint32_t flags = 0;
    std::vector<Slot> slots;
    CopyPool copies;
};

namespace {

void free_slots(aesgpu_pipeline *pl) {
    for (Slot &s : pl->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.d_in) (void)hipFree(s.d_in);
        if (s.d_out) (void)hipFree(s.d_out);
        if (s.h_in) (void)hipHostFree(s.h_in);
        if (s.h_out) (void)hipHostFree(s.h_out);
        s = Slot{};
    }
}

// Waits for a slot's chunk and copies its staged output to the caller.
int finish(aesgpu_pipeline *pl, Slot &s, uint8_t *h_out) {
    if (!s.busy) return AESGPU_OK;
    s.busy = false;
    if (hipEventSynchronize(s.done) != hipSuccess) return AESGPU_EHIP;
    if (s.staged_out) pl->copies.copy(h_out + s.off, s.h_out, s.len);
    return AESGPU_OK;
}

// Pinned, mapped host memory and its device address.
bool alloc_mapped(size_t n, void **host, void **dev) {
    if (hipHostMalloc(host, n, hipHostMallocMapped | hipHostMallocPortable) != hipSuccess ||
        !*host)
        return false;
    return hipHostGetDevicePointer(dev, *host, 0) == hipSuccess && *dev;
}

// The device call for one chunk of `op` starting at byte `off` of the run.
int launch_chunk(aesgpu_ctx *ctx, const aesgpu_key *key, const aesgpu_host_op &op,
                 const uint8_t *h_in, uint64_t off, const void *d_in, void *d_out, uint64_t len,
                 hipStream_t st) {
    auto *stream = reinterpret_cast<aesgpu_stream_t>(st);
    const uint64_t first_block = off / 16;
    switch (op.op) {
        case AESGPU_OP_ECB_ENCRYPT:
            return aesgpu_ecb_encrypt(ctx, key, d_in, d_out, len / 16, stream);
        case AESGPU_OP_ECB_DECRYPT:
            return aesgpu_ecb_decrypt(ctx, key, d_in, d_out, len / 16, stream);
        case AESGPU_OP_CTR:
            return aesgpu_ctr_xcrypt(ctx, key, op.nonce, uint32_t(op.ctr0 + first_block), d_in,
                                     d_out, len, stream);
        case AESGPU_OP_CTR_LE128:
            return aesgpu_ctr_le128_xcrypt(ctx, key, op.iv, first_block, d_in, d_out, len, stream);
        case AESGPU_OP_CBC_DECRYPT:
            // Eq. (2) across chunks: a chunk's IV is the previous ciphertext
            // block, read from the caller's input.
            return aesgpu_cbc_decrypt(ctx, key, off == 0 ? op.iv : h_in + off - 16, d_in, d_out,
                                      len / 16, stream);
    }
    return AESGPU_EINVAL;
}

}  // namespace

extern "C" {

int aesgpu_host_alloc(size_t n_bytes, void **out) {
    if (!out || n_bytes == 0) return AESGPU_EINVAL;
    *out = nullptr;
    void *p = nullptr, *d = nullptr;
    if (hipHostMalloc(&p, n_bytes, hipHostMallocMapped | hipHostMallocPortable) != hipSuccess ||
        !p) {
        (void)hipGetLastError();
        return AESGPU_ENOMEM;
    }
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess || !d) {
        (void)hipGetLastError();
        (void)hipHostFree(p);
        return AESGPU_EHIP;
    }
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    g_pinned[reinterpret_cast<uintptr_t>(p)] = {n_bytes, reinterpret_cast<uintptr_t>(d)};
    *out = p;
    return AESGPU_OK;
}

int aesgpu_host_free(void *p) {
    if (!p) return AESGPU_OK;
    {
        std::lock_guard<std::mutex> lk(g_pinned_mu);
        auto it = g_pinned.find(reinterpret_cast<uintptr_t>(p));
        if (it == g_pinned.end()) return AESGPU_EINVAL;
        g_pinned.erase(it);
    }
    return hipHostFree(p) == hipSuccess ? AESGPU_OK : AESGPU_EHIP;
}

int aesgpu_pipeline_create(aesgpu_ctx *ctx, size_t chunk_bytes, int n_slots, uint32_t flags,
                           aesgpu_pipeline **out) {
    if (!out) return AESGPU_EINVAL;
    *out = nullptr;
    if (!ctx || (flags & ~uint32_t(AESGPU_PIPELINE_COPY))) return AESGPU_EINVAL;
    if (chunk_bytes == 0) chunk_bytes = kDefaultChunk;
    if (n_slots == 0) n_slots = kDefaultSlots;
    if (chunk_bytes % 16 != 0 || n_slots < 1 || n_slots > kMaxSlots) return AESGPU_EINVAL;
    aesgpu_pipeline *pl = nullptr;
    try {
        pl = new aesgpu_pipeline;
    } catch (...) {
        return AESGPU_ENOMEM;
    }
    pl->ctx = ctx;
    pl->device = ctx->device;
    pl->chunk = chunk_bytes;
    pl->flags = flags;
    pl->slots.resize(size_t(n_slots));
    DeviceGuard g(ctx->device);
    int st = g.ok() ? AESGPU_OK : AESGPU_EHIP;
    for (Slot &s : pl->slots) {
        if (st != AESGPU_OK) break;
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
            st = AESGPU_EHIP;
        } else if (!alloc_mapped(chunk_bytes, &s.h_in, &s.hd_in) ||
                   !alloc_mapped(chunk_bytes, &s.h_out, &s.hd_out) ||
                   ((flags & AESGPU_PIPELINE_COPY) &&
                    (hipMalloc(&s.d_in, chunk_bytes) != hipSuccess ||
                     hipMalloc(&s.d_out, chunk_bytes) != hipSuccess))) {
            st = AESGPU_ENOMEM;
        }
    }
    if (st != AESGPU_OK) {
        (void)hipGetLastError();
        free_slots(pl);
        delete pl;
        return st;
    }
    *out = pl;
    return AESGPU_OK;
}

int aesgpu_pipeline_run(aesgpu_pipeline *pl, const aesgpu_key *key, const aesgpu_host_op *op,
                        const void *h_in, void *h_out, size_t n_bytes) {
    if (!pl || !key_ok(key) || !op) return AESGPU_EINVAL;
    if (op->op > AESGPU_OP_CBC_DECRYPT) return AESGPU_EINVAL;
    if (n_bytes == 0) return AESGPU_OK;
    if (!h_in || !h_out) return AESGPU_EINVAL;
    const bool whole_blocks = op->op == AESGPU_OP_ECB_ENCRYPT ||
                              op->op == AESGPU_OP_ECB_DECRYPT || op->op == AESGPU_OP_CBC_DECRYPT;
    if (whole_blocks && n_bytes % 16 != 0) return AESGPU_EINVAL;
    if (h_in != h_out && ranges_overlap(h_in, h_out, n_bytes)) return AESGPU_EINVAL;
    if (op->op == AESGPU_OP_CBC_DECRYPT && h_in == h_out) return AESGPU_EINVAL;
    if (op->op == AESGPU_OP_CTR &&
        uint64_t(op->ctr0) + (uint64_t(n_bytes) + 15) / 16 - 1 > 0xFFFFFFFFull)
        return AESGPU_ECTR_OVERFLOW;

    DeviceGuard g(pl->device);
    if (!g.ok()) return AESGPU_EHIP;
    const auto *src = static_cast<const uint8_t *>(h_in);
    auto *dst = static_cast<uint8_t *>(h_out);
    const uintptr_t dev_in = pinned_device_address(h_in, n_bytes);
    const uintptr_t dev_out = pinned_device_address(h_out, n_bytes);
    const bool pinned_in = dev_in != 0, pinned_out = dev_out != 0;
    if (pinned_in && pinned_out && !(pl->flags & AESGPU_PIPELINE_COPY) && dev_in % 16 == 0 &&
        dev_out % 16 == 0) {
        // Zero copy: one kernel reads and writes host memory over the link.
        Slot &s = pl->slots[0];
        int zs = launch_chunk(pl->ctx, key, *op, src, 0, reinterpret_cast<const void *>(dev_in),
                              reinterpret_cast<void *>(dev_out), n_bytes, s.stream);
        if (zs == AESGPU_OK && hipStreamSynchronize(s.stream) != hipSuccess) zs = AESGPU_EHIP;
        if (zs != AESGPU_OK) (void)hipGetLastError();
        return zs;
    }
    const size_t n_slots = pl->slots.size();
    const bool dma = pl->flags & AESGPU_PIPELINE_COPY;
    // Without DMA copies the kernel works on host memory: the caller's own
    // pinned range where it is 16-byte aligned (chunk offsets keep that),
    // else the slot's staging buffer.
    const bool direct_in = !dma && pinned_in && dev_in % 16 == 0;
    const bool direct_out = !dma && pinned_out && dev_out % 16 == 0;
    int st = AESGPU_OK;
    uint64_t c = 0;
    for (uint64_t off = 0; off < n_bytes && st == AESGPU_OK; off += pl->chunk, ++c) {
        Slot &s = pl->slots[c % n_slots];
        st = finish(pl, s, dst);
        if (st != AESGPU_OK) break;
        const uint64_t len = std::min<uint64_t>(pl->chunk, n_bytes - off);
        const void *k_in;
        void *k_out;
        if (dma) {
            const void *from = src + off;
            if (!pinned_in) {
                pl->copies.copy(s.h_in, src + off, len);
                from = s.h_in;
            }
            if (hipMemcpyAsync(s.d_in, from, len, hipMemcpyHostToDevice, s.stream) !=
                hipSuccess) {
                st = AESGPU_EHIP;
                break;
            }
            k_in = s.d_in;
            k_out = s.d_out;
        } else {
            if (direct_in) {
                k_in = reinterpret_cast<const void *>(dev_in + off);
            } else {
                pl->copies.copy(s.h_in, src + off, len);
                k_in = s.hd_in;
            }
            k_out = direct_out ? reinterpret_cast<void *>(dev_out + off) : s.hd_out;
        }
        st = launch_chunk(pl->ctx, key, *op, src, off, k_in, k_out, len, s.stream);
        if (st != AESGPU_OK) break;
        if (dma) {
            s.staged_out = !pinned_out;
            void *to = pinned_out ? static_cast<void *>(dst + off) : s.h_out;
            if (hipMemcpyAsync(to, s.d_out, len, hipMemcpyDeviceToHost, s.stream) != hipSuccess) {
                st = AESGPU_EHIP;
                break;
            }
        } else {
            s.staged_out = !direct_out;
        }
        if (hipEventRecord(s.done, s.stream) != hipSuccess) {
            st = AESGPU_EHIP;
            break;
        }
        s.busy = true;
        s.off = off;
        s.len = len;
    }
    // Drain in issue order (so staged copies land before the call returns).
    for (uint64_t k = 0; k < n_slots; ++k) {
        const int fs = finish(pl, pl->slots[(c + k) % n_slots], dst);
        if (st == AESGPU_OK) st = fs;
    }
    if (st != AESGPU_OK) {
        // A chunk that failed part way may have left a copy or a kernel on
        // its stream that no event covers; none may touch the caller's
        // buffers after the call returns.
        for (Slot &s : pl->slots) (void)hipStreamSynchronize(s.stream);
        (void)hipGetLastError();
    }
    return st;
}

void aesgpu_pipeline_destroy(aesgpu_pipeline *pl) {
    if (!pl) return;
    DeviceGuard g(pl->device);
    free_slots(pl);
    delete pl;
}

}  // extern "C"
