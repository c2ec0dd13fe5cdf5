// Host-staged pipeline: host buffers in, host buffers out.
//
// The paper's section 3 moves every buffer across the bus: the input is
// mapped into a texture, drawn, and the output read back, and its section 3.1
// finds the GPU slower than the CPU for small data because of that transfer
// cost.  This is the same data path done as a pipeline: the buffer is cut
// into chunks, and each chunk's host-to-device copy, kernel and device-to-host
// copy run on one of several streams, so the copies of one chunk overlap the
// kernels and copies of the others.  Pageable host memory goes through pinned
// staging buffers with a CPU copy, which overlaps the device work of the
// other slots.  Host buffers allocated with aesgpu_host_alloc() (pinned and
// mapped into the device's address space) need no staging: by default the
// kernel then reads its input from and writes its output to host memory
// directly over PCIe (zero copy), so both directions of the link are busy at
// once; with AESGPU_PIPELINE_COPY they are moved by DMA copies instead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
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
    void *d_in = nullptr, *d_out = nullptr;
    void *h_in = nullptr, *h_out = nullptr;   // pinned staging
    bool busy = false;
    uint64_t off = 0, len = 0;                // chunk in flight
    bool staged_out = false;
};

}  // namespace

struct aesgpu_pipeline {
    aesgpu_ctx *ctx = nullptr;
    int device = 0;
    size_t chunk = 0;
    uint32_t flags = 0;
    std::vector<Slot> slots;
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
int finish(Slot &s, uint8_t *h_out) {
    if (!s.busy) return AESGPU_OK;
    s.busy = false;
    if (hipEventSynchronize(s.done) != hipSuccess) return AESGPU_EHIP;
    if (s.staged_out) std::memcpy(h_out + s.off, s.h_out, s.len);
    return AESGPU_OK;
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
    auto *pl = new (std::nothrow) aesgpu_pipeline;
    if (!pl) return AESGPU_ENOMEM;
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
        } else if (hipMalloc(&s.d_in, chunk_bytes) != hipSuccess ||
                   hipMalloc(&s.d_out, chunk_bytes) != hipSuccess ||
                   hipHostMalloc(&s.h_in, chunk_bytes, hipHostMallocDefault) != hipSuccess ||
                   hipHostMalloc(&s.h_out, chunk_bytes, hipHostMallocDefault) != hipSuccess) {
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
    int st = AESGPU_OK;
    uint64_t c = 0;
    for (uint64_t off = 0; off < n_bytes && st == AESGPU_OK; off += pl->chunk, ++c) {
        Slot &s = pl->slots[c % n_slots];
        st = finish(s, dst);
        if (st != AESGPU_OK) break;
        const uint64_t len = std::min<uint64_t>(pl->chunk, n_bytes - off);
        const void *from = src + off;
        if (!pinned_in) {
            std::memcpy(s.h_in, src + off, len);
            from = s.h_in;
        }
        if (hipMemcpyAsync(s.d_in, from, len, hipMemcpyHostToDevice, s.stream) != hipSuccess) {
            st = AESGPU_EHIP;
            break;
        }
        st = launch_chunk(pl->ctx, key, *op, src, off, s.d_in, s.d_out, len, s.stream);
        if (st != AESGPU_OK) break;
        s.staged_out = !pinned_out;
        void *to = pinned_out ? static_cast<void *>(dst + off) : s.h_out;
        if (hipMemcpyAsync(to, s.d_out, len, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
            hipEventRecord(s.done, s.stream) != hipSuccess) {
            st = AESGPU_EHIP;
            break;
        }
        s.busy = true;
        s.off = off;
        s.len = len;
    }
    // Drain in issue order (so staged copies land before the call returns).
    for (uint64_t k = 0; k < n_slots; ++k) {
        const int fs = finish(pl->slots[(c + k) % n_slots], dst);
        if (st == AESGPU_OK) st = fs;
    }
    if (st != AESGPU_OK) (void)hipGetLastError();
    return st;
}

void aesgpu_pipeline_destroy(aesgpu_pipeline *pl) {
    if (!pl) return;
    DeviceGuard g(pl->device);
    free_slots(pl);
    delete pl;
}

}  // extern "C"
