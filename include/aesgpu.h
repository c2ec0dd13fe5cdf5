/*
 * aesgpu.h -- C ABI of the MI355X (gfx950) AES block-encryption library.
 *
 * The library encrypts and decrypts buffers that already live in device
 * memory, with the round structure of the paper's section 2.1: the state is
 * four 32-bit words and SubBytes, ShiftRows and MixColumns are fused into four
 * 32-bit lookup tables T0..T3 (Eq. (1)), plus AddRoundKey; decryption uses the
 * inverse tables.  The paper's parallel modes (section 3) are ECB and CTR for
 * both directions and CBC for decryption only (Eq. (2)).  Key expansion and
 * the block cipher itself are the ones the paper defers to FIPS-197.
 *
 * Conventions used by every call:
 *
 *  - Status: every int-returning call returns AESGPU_OK (0) or a negative
 *    AESGPU_E* code.  aesgpu_strerror() names a code.
 *  - Byte order: a block is the byte sequence in[0..15]; the state is
 *    s[r][c] = in[r + 4c].  Words are little-endian: 32-bit word c of a block
 *    is column c and its byte k is row k, the paper's I_{c,k}.
 *  - Device buffers (`d_in`, `d_out`) are caller-owned device pointers, 16-byte
 *    aligned (AESGPU_EALIGN otherwise).  d_in == d_out (in place) is allowed;
 *    any other overlap is AESGPU_EINVAL.  A zero length is a no-op returning
 *    AESGPU_OK without touching the device.
 *  - Streams: `stream` is a HIP stream (hipStream_t; NULL is the null
 *    stream).  Calls only enqueue work: they return once the launch is queued,
 *    and faults inside the kernel surface at the next synchronisation.
 *  - Errors: argument errors are detected on the host, in the order the
 *    arguments appear, before any HIP call.  A failed launch returns
 *    AESGPU_EHIP.
 *  - Threads: a context is immutable after aesgpu_create(); calls on one
 *    context from several host threads and streams may run concurrently.
 */
#ifndef AESGPU_H
#define AESGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same underlying type as hipStream_t. */
typedef struct ihipStream_t *aesgpu_stream_t;

enum {
    AESGPU_OK = 0,
    AESGPU_EINVAL = -1,        /* bad argument (NULL, bad enum, overlap, ...) */
    AESGPU_EKEYLEN = -2,       /* key length not 16, 24 or 32 bytes */
    AESGPU_EALIGN = -3,        /* device pointer not 16-byte aligned */
    AESGPU_ECTR_OVERFLOW = -4, /* 32-bit block counter would wrap */
    AESGPU_ENOMEM = -5,        /* device or host allocation failed */
    AESGPU_EHIP = -6,          /* a HIP runtime call or launch failed */
    AESGPU_EAGAIN = -7,        /* server full: retry after polling */
    AESGPU_ESCRATCH = -8       /* batch larger than the fixed scratch of
                                  aesgpu_batch_run_noalloc() */
};

typedef struct aesgpu_ctx aesgpu_ctx;

/*
 * Expanded key: caller-owned plain data, filled by aesgpu_expand_key() and
 * passed by pointer to the buffer calls (its words travel to the GPU as
 * kernel arguments, so it may be reused or freed as soon as a call returns).
 *   enc[4r + c] = round key r, column c, as a little-endian word (FIPS-197
 *                 KeyExpansion), r = 0..nr.
 *   dec[4r + c] = round keys of the equivalent inverse cipher: dec round r is
 *                 InvMixColumns(enc round nr - r) for 0 < r < nr, and the
 *                 plain enc rounds nr and 0 at r = 0 and r = nr.
 */
typedef struct {
    uint32_t key_bits; /* 128, 192 or 256 */
    uint32_t nr;       /* 10, 12 or 14 rounds */
    uint32_t enc[60];
    uint32_t dec[60];
} aesgpu_key;

/*
 * Creates a context on HIP device `device`: builds the lookup tables T0..T3,
 * their inverses and the S-boxes on the host and copies them to the device
 * once (the paper's section 3 creates all resources once at start-up).
 * *out receives the context.  The single-buffer calls choose their blocks per
 * lane by size (and CBC decryption with 192- or 256-bit keys takes at most 2);
 * the environment variable AESGPU_FORCE_BPL=1, 2 or 4, read here, fixes it
 * for this context's calls (for tests and measurements).  A single-buffer
 * call of more than 4095 tiles per CU (about 64 GiB at 4 blocks per lane on
 * 256 CUs) runs as several launches on the same stream;
 * AESGPU_MAX_TILES_PER_CU=2..4096, read here, lowers that limit (for tests).
 * Errors: EINVAL (out NULL, bad device), ENOMEM, EHIP.
 */
int aesgpu_create(aesgpu_ctx **out, int device);

/* Frees the context's device tables.  NULL is ignored.  The caller must make
 * sure no launch that uses the context is still running. */
void aesgpu_destroy(aesgpu_ctx *ctx);

/*
 * Host-side key expansion (FIPS-197 KeyExpansion, which the paper's section
 * 2.1 defers to): key_bytes = 16, 24 or 32 gives 10, 12 or 14 rounds.
 * Fills *out.  Errors: EINVAL (NULL), EKEYLEN.  Touches no device.
 */
int aesgpu_expand_key(const uint8_t *key, size_t key_bytes, aesgpu_key *out);

/*
 * ECB encryption of n_blocks 16-byte blocks (section 2.1 Eq. (1) rounds per
 * block; ECB is one of the parallel modes of section 3): d_out[i] =
 * E_K(d_in[i]).  Padding is the caller's (the paper leaves the scheme open).
 * Errors: EINVAL (ctx or key NULL, key not expanded, NULL buffer with n > 0,
 * partial overlap), EALIGN, EHIP.
 */
int aesgpu_ecb_encrypt(aesgpu_ctx *ctx, const aesgpu_key *key, const void *d_in, void *d_out,
                       size_t n_blocks, aesgpu_stream_t stream);

/* ECB decryption with the inverse tables: d_out[i] = D_K(d_in[i]).  Same
 * arguments and errors as aesgpu_ecb_encrypt(). */
int aesgpu_ecb_decrypt(aesgpu_ctx *ctx, const aesgpu_key *key, const void *d_in, void *d_out,
                       size_t n_blocks, aesgpu_stream_t stream);

/*
 * CTR mode (section 3), the same call for encryption and decryption:
 * block i's keystream is E_K(nonce[0..11] || BE32(ctr0 + i)) and
 * d_out = d_in XOR keystream over n_bytes, which need not be a multiple of 16
 * (the last keystream block is cut).  The counter never wraps: if
 * ctr0 + ceil(n_bytes / 16) - 1 > 2^32 - 1 the call returns ECTR_OVERFLOW.
 * nonce is a host pointer to 12 bytes.  Errors: EINVAL, EALIGN,
 * ECTR_OVERFLOW, EHIP.
 */
int aesgpu_ctr_xcrypt(aesgpu_ctx *ctx, const aesgpu_key *key, const uint8_t *nonce, uint32_t ctr0,
                      const void *d_in, void *d_out, size_t n_bytes, aesgpu_stream_t stream);

/*
 * CTR mode with the paper's own counter (section 3 listing): block i's
 * counter is the 16-byte IV read as a little-endian 128-bit integer plus
 * (index0 + i), modulo 2^128.  iv is a host pointer to 16 bytes.  Any length;
 * never fails for overflow (the 128-bit add wraps by definition).
 * Errors: EINVAL, EALIGN, EHIP.
 */
int aesgpu_ctr_le128_xcrypt(aesgpu_ctx *ctx, const aesgpu_key *key, const uint8_t *iv,
                            uint64_t index0, const void *d_in, void *d_out, size_t n_bytes,
                            aesgpu_stream_t stream);

/*
 * CBC decryption, section 3 Eq. (2): d_out[i] = D_K(d_in[i]) XOR d_in[i-1],
 * with d_in[-1] = iv (host pointer to 16 bytes).  Unlike the paper, the first
 * block's XOR is done on the GPU too.  Not in place: d_in and d_out must not
 * overlap (EINVAL), since every block reads its predecessor's ciphertext.
 * Errors: EINVAL, EALIGN, EHIP.
 */
int aesgpu_cbc_decrypt(aesgpu_ctx *ctx, const aesgpu_key *key, const uint8_t *iv,
                       const void *d_in, void *d_out, size_t n_blocks, aesgpu_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Batched messages: one persistent launch per table set                     */
/* ------------------------------------------------------------------------ */

enum { AESGPU_MODE_ECB = 0, AESGPU_MODE_CTR = 1, AESGPU_MODE_CBC = 2 };
enum { AESGPU_DIR_ENCRYPT = 0, AESGPU_DIR_DECRYPT = 1 };

/*
 * One message of a batch (host struct, 48 bytes).  Its input is
 * d_in + in_off and its output d_out + out_off (both 16-byte aligned), its key
 * the raw key bytes at d_keys + 32 * key_slot.  ECB messages are whole blocks
 * and use `dir`; CTR messages (nonce || BE32(ctr0 + i), as
 * aesgpu_ctr_xcrypt()) may end in a partial block and ignore `dir`.  CBC
 * messages (section 3, Eq. (2)) are whole blocks and use `dir`; their 16-byte
 * IV is the 16 bytes starting at `nonce` (nonce[0..11], then ctr0's bytes in
 * memory order).  CBC decryption is block-parallel; CBC encryption is
 * sequential within a message (the paper leaves it out for one stream), so a
 * batch runs up to 16 such messages of one key size per wave, four lanes per
 * message, in a launch of its own after the persistent one, and only batches
 * of many short CBC-encrypt messages use the GPU well.
 */
typedef struct {
    uint64_t in_off;
    uint64_t out_off;
    uint64_t n_bytes;
    uint32_t key_slot;
    uint16_t key_bits;   /* 128, 192 or 256 */
    uint8_t mode;        /* AESGPU_MODE_ECB or AESGPU_MODE_CTR */
    uint8_t dir;         /* AESGPU_DIR_ENCRYPT or AESGPU_DIR_DECRYPT */
    uint8_t nonce[12];
    uint32_t ctr0;
} aesgpu_msg;

#define AESGPU_BATCH_NO_GRAPH 1u /* enqueue the launches directly, no hipGraph */

/* Launch shape of a batch; zero fields take the defaults (4 blocks per lane,
 * 8192-block tiles).  tile_blocks must be a multiple of 64 * blocks_per_lane. */
typedef struct {
    uint32_t blocks_per_lane; /* 1, 2 or 4 */
    uint32_t tile_blocks;
    uint32_t flags;           /* AESGPU_BATCH_* */
} aesgpu_batch_config;

typedef struct {
    uint64_t n_msgs;
    uint64_t n_tiles_forward;  /* ECB-encrypt and CTR tiles */
    uint64_t n_tiles_inverse;  /* ECB-decrypt tiles */
    uint64_t total_bytes;      /* sum of n_bytes */
    uint64_t in_bytes_needed;  /* max(in_off + n_bytes) */
    uint64_t out_bytes_needed; /* max(out_off + n_bytes) */
    uint32_t blocks_per_lane;
    uint32_t tile_blocks;
    uint32_t launches;         /* launches per run: 1 persistent launch (if any ECB, CTR or
                                  CBC-decrypt blocks) + 1 if any CBC-encrypt messages */
} aesgpu_batch_stats;

typedef struct aesgpu_batch aesgpu_batch;

/*
 * Plans a batch of m messages (the paper's per-pixel independence, section 3,
 * applied across messages): validates every message, cuts them into
 * message-pure tiles, sorts each queue longest first and copies the
 * descriptors to the device (synchronously).  cfg may be NULL.  The plan
 * holds device memory until aesgpu_batch_free().  Errors: EINVAL (bad mode,
 * direction, config, ECB length not a multiple of 16), EKEYLEN (key_bits),
 * EALIGN (offsets), ECTR_OVERFLOW, ENOMEM, EHIP.
 */
int aesgpu_batch_plan(aesgpu_ctx *ctx, const aesgpu_msg *msgs, size_t m,
                      const aesgpu_batch_config *cfg, aesgpu_batch **out);

/*
 * Runs a planned batch on `stream`: every message is encrypted or decrypted
 * with its own key, expanded on the device inside the launch (FIPS-197
 * KeyExpansion, plus the equivalent-inverse-cipher keys for decryption).
 * d_keys holds n_key_slots raw keys at a 32-byte stride (key bytes first);
 * d_in and d_out are in_bytes / out_bytes long and must hold every message
 * (EINVAL otherwise).  d_in == d_out runs in place, except that a CBC-decrypt
 * message whose input and output ranges meet is then EINVAL (each block
 * reads its predecessor's ciphertext); other overlap of d_in and d_out is
 * EINVAL.  Messages whose outputs overlap each other, or overlap a
 * CBC-decrypt message's input, give undefined output.  By
 * default the launches are captured once into a hipGraph and replayed; the
 * graph is re-captured when d_keys, d_in or d_out change.  On ROCm 7 a
 * replay costs 5-9 us more than launching the same kernels directly, which
 * matters only for small batches: plan those with AESGPU_BATCH_NO_GRAPH when
 * latency counts.  Calls on one plan must not overlap in time (they share
 * the plan's tile counters, which every run leaves at zero).
 * Errors: EINVAL, EALIGN, EHIP.
 */
int aesgpu_batch_run(aesgpu_batch *plan, const uint8_t *d_keys, size_t n_key_slots,
                     const void *d_in, size_t in_bytes, void *d_out, size_t out_bytes,
                     aesgpu_stream_t stream);

/*
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): plans and runs one batch in a single call
 * and allocates no device memory.  Messages, keys, buffers, stream and cfg
 * mean what they mean for aesgpu_batch_plan() and aesgpu_batch_run(), with the
 * same errors; the launches are enqueued directly (no hipGraph).  The batch's
 * device descriptors (64 bytes per message, 16 per tile, the queue counters
 * and the CBC-encryption groups) go to a fixed scratch area of
 * AESGPU_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends; a batch needing more returns AESGPU_ESCRATCH before any
 * HIP call (65,536 messages of up to 1 MiB in 8192-block tiles need about
 * 6 MB).  The descriptors are built on the host and copied on `stream` from
 * pageable host memory (a copy that completes before the call returns).
 * Every call on one GPU uses that GPU's one scratch area: calls whose runs
 * overlap in time on one GPU (other streams, other contexts, other threads)
 * race and give undefined output; serialise them, for instance on one
 * stream.  Errors: EINVAL, EKEYLEN, EALIGN, ECTR_OVERFLOW, ESCRATCH, EHIP.
 */
#define AESGPU_NOALLOC_SCRATCH_BYTES (8u << 20)
int aesgpu_batch_run_noalloc(aesgpu_ctx *ctx, const aesgpu_msg *msgs, size_t m,
                             const aesgpu_batch_config *cfg, const uint8_t *d_keys,
                             size_t n_key_slots, const void *d_in, size_t in_bytes, void *d_out,
                             size_t out_bytes, aesgpu_stream_t stream);

/* Plan statistics (host only).  Errors: EINVAL. */
int aesgpu_batch_info(const aesgpu_batch *plan, aesgpu_batch_stats *out);

/* Frees the plan (device descriptors, graph).  NULL is ignored.  The caller
 * must make sure no run of the plan is still executing. */
void aesgpu_batch_free(aesgpu_batch *plan);

/* ------------------------------------------------------------------------ */
/* Host-staged pipeline: host buffers in, host buffers out                   */
/* ------------------------------------------------------------------------ */

/*
 * Pinned host memory, mapped into the device's address space, that
 * aesgpu_pipeline_run() recognises (no staging copy).  *out receives the host
 * pointer.  Errors: EINVAL (out NULL, zero size), ENOMEM, EHIP.
 * aesgpu_host_free() takes only pointers returned here (EINVAL otherwise;
 * NULL is ignored).
 */
int aesgpu_host_alloc(size_t n_bytes, void **out);
int aesgpu_host_free(void *p);

enum {
    AESGPU_OP_ECB_ENCRYPT = 0,
    AESGPU_OP_ECB_DECRYPT = 1,
    AESGPU_OP_CTR = 2,          /* nonce || BE32(ctr0 + i), as aesgpu_ctr_xcrypt() */
    AESGPU_OP_CTR_LE128 = 3,    /* iv + i as a 128-bit LE integer, as aesgpu_ctr_le128_xcrypt() */
    AESGPU_OP_CBC_DECRYPT = 4   /* Eq. (2) with iv, as aesgpu_cbc_decrypt() */
};

/* One mode call over a host buffer (host struct). */
typedef struct {
    uint32_t op;        /* AESGPU_OP_* */
    uint32_t ctr0;      /* AESGPU_OP_CTR */
    uint8_t nonce[12];  /* AESGPU_OP_CTR */
    uint8_t iv[16];     /* AESGPU_OP_CTR_LE128, AESGPU_OP_CBC_DECRYPT */
} aesgpu_host_op;

typedef struct aesgpu_pipeline aesgpu_pipeline;

#define AESGPU_PIPELINE_COPY 1u /* move aesgpu_host_alloc() memory by DMA copies, not zero copy */

/*
 * The data path of the paper's section 3 (upload, encrypt, read back), as a
 * pipeline: chunk_bytes (a multiple of 16; 0 = 8 MiB) per chunk and n_slots
 * chunks in flight (1..16; 0 = 3), each slot with its own stream and two
 * pinned, mapped staging buffers (plus two device chunk buffers with
 * AESGPU_PIPELINE_COPY), allocated here, and a few host threads that split
 * the staging copies.  flags: 0 or AESGPU_PIPELINE_COPY.  Errors: EINVAL,
 * ENOMEM, EHIP.
 */
int aesgpu_pipeline_create(aesgpu_ctx *ctx, size_t chunk_bytes, int n_slots, uint32_t flags,
                           aesgpu_pipeline **out);

/*
 * Runs `op` over n_bytes from host memory h_in to host memory h_out and
 * returns when the output is complete.  When both ranges lie in
 * aesgpu_host_alloc() allocations (and AESGPU_PIPELINE_COPY is not set), the
 * library's kernel for `op` reads and writes them directly over the host link
 * (zero copy, both directions at once), in one launch.  Otherwise the buffer
 * runs in chunks, one per slot and stream at a time (chunk k continues the
 * counter or the CBC chain of chunk k - 1).  Without AESGPU_PIPELINE_COPY
 * the kernel still works on host memory: an aligned aesgpu_host_alloc()
 * range directly, other memory through the slot's staging buffers (a CPU
 * copy in before the kernel and out after it).  With AESGPU_PIPELINE_COPY
 * each chunk is copied to the device by DMA, processed and copied back
 * (pageable memory through the staging buffers).
 * h_in == h_out runs in place (not for CBC); other overlap is EINVAL.  ECB
 * and CBC take whole blocks.  Calls on one pipeline must not overlap in time.
 * Errors: EINVAL, ECTR_OVERFLOW, EHIP.
 */
int aesgpu_pipeline_run(aesgpu_pipeline *pl, const aesgpu_key *key, const aesgpu_host_op *op,
                        const void *h_in, void *h_out, size_t n_bytes);

/* Frees the pipeline's buffers and streams (waits for its work).  NULL is
 * ignored. */
void aesgpu_pipeline_destroy(aesgpu_pipeline *pl);

/* ------------------------------------------------------------------------ */
/* Device-memory range allocator (host bookkeeping only)                    */
/* ------------------------------------------------------------------------ */

/*
 * Best-fit allocator of byte ranges [0, capacity) with coalescing on
 * release, in multiples of `granule` (a power of two dividing capacity): an
 * allocation takes the start of the smallest free range that fits (the
 * lowest offset among equal sizes), in O(log n) for n free ranges.  It
 * only does the bookkeeping (no device memory is touched); the server admits
 * requests with it.  Not thread-safe.  Errors: EINVAL (bad sizes, a release
 * that is not a live allocation), ENOMEM; aesgpu_arena_alloc returns EAGAIN
 * when no free range is large enough right now and EINVAL when the request
 * exceeds the capacity.
 */
typedef struct aesgpu_arena aesgpu_arena;
int aesgpu_arena_create(uint64_t capacity, uint64_t granule, aesgpu_arena **out);
int aesgpu_arena_alloc(aesgpu_arena *arena, uint64_t n_bytes, uint64_t *offset);
int aesgpu_arena_release(aesgpu_arena *arena, uint64_t offset, uint64_t n_bytes);
int aesgpu_arena_query(const aesgpu_arena *arena, uint64_t *used, uint64_t *largest_free,
                       uint64_t *high_water);
void aesgpu_arena_destroy(aesgpu_arena *arena);

/* ------------------------------------------------------------------------ */
/* Continuous-batching server                                               */
/* ------------------------------------------------------------------------ */

typedef struct aesgpu_server aesgpu_server;

typedef struct {
    uint64_t arena_bytes;        /* device memory for request outputs (multiple of 256) */
    uint32_t n_streams;          /* batches in flight at once (0 = 4, at most 8) */
    uint32_t blocks_per_lane;    /* 1, 2 or 4 (0 = 2) */
    uint32_t tile_blocks;        /* 0 = chosen per batch (about two tiles per wave slot) */
    uint32_t max_batch_requests; /* 0 = no limit */
    uint64_t max_batch_bytes;    /* 0 = no limit */
    uint32_t max_queued;         /* waiting requests before EAGAIN (0 = 2^20) */
    uint32_t direct_requests;    /* batches of at most this many requests, with none
                                    waiting behind them, run as one single-buffer launch
                                    per request (0 = 4, at most 16;
                                    AESGPU_SERVER_NO_DIRECT: always the batched kernel) */
    uint32_t flags;              /* 0 or AESGPU_SERVER_RESIDENT */
} aesgpu_server_config;

#define AESGPU_SERVER_NO_DIRECT 0xFFFFFFFFu
#define AESGPU_SERVER_RESIDENT 1u   /* one kernel stays on the GPU and takes the tiles */

/* A finished request.  d_out points into the server's arena and stays valid
 * until aesgpu_server_release().  Times are seconds on the server clock
 * (aesgpu_server_now()). */
typedef struct {
    uint64_t req_id;
    int32_t status;     /* AESGPU_OK or the error that failed its batch */
    uint32_t reserved;
    void *d_out;
    uint64_t n_bytes;
    double t_arrival;   /* as passed to submit */
    double t_launch;    /* its batch was enqueued */
    double t_done;      /* its batch was seen complete */
} aesgpu_done;

/* One request of a replayed arrival trace (t_arrival relative to t_start). */
typedef struct {
    uint64_t req_id;    /* 0 .. n-1, each once */
    double t_arrival;
    const void *d_in;
    uint64_t n_bytes;
    uint32_t key_id;
    uint32_t dir;       /* AESGPU_DIR_ENCRYPT or AESGPU_DIR_DECRYPT */
} aesgpu_request;

typedef struct {
    uint64_t batches;
    uint64_t requests_submitted;
    uint64_t requests_done;
    uint64_t bytes_done;
    uint64_t max_batch_requests;
    uint64_t queued;             /* waiting for admission now */
    uint64_t arena_used;
    uint64_t arena_high_water;
    uint64_t rebalances;         /* resident mode: kernel stops that changed the split
                                    of workgroups between encryption and decryption */
} aesgpu_server_stats;

/*
 * Starts a server on ctx's device: expands the n_keys pool keys (raw bytes at
 * a 32-byte stride in host memory `keys`, sizes in key_bits) and keeps their
 * encryption and decryption schedules resident on the device, allocates the
 * output arena and the streams, and starts the dispatcher thread.  Requests
 * are ECB (the paper's section 3 parallel mode) in either direction.  Each
 * dispatch launches all admitted requests as one batched run (the persistent
 * launch of aesgpu_batch_run, with resident schedules instead of device key
 * expansion, after an upload of the batch's descriptors); a batch of at most
 * direct_requests requests, when no other request is waiting, instead runs as
 * one single-buffer kernel per request with the round keys as kernel
 * arguments, which saves the upload.
 *
 * With AESGPU_SERVER_RESIDENT in flags there are no per-batch launches: one
 * kernel stays on the GPU (one workgroup per CU, half of them holding the
 * encryption tables and half the decryption tables) and takes tiles from two
 * rings in pinned host memory, which the dispatcher fills as it admits
 * requests (tiles sized so that a request spreads over the waves that the
 * requests already in flight leave free).  The kernel reports each finished
 * request through a completion ring in pinned memory.  When a large backlog
 * (a quarter millisecond of the chip or more) leans to one direction by at
 * least an eighth of the chip, the dispatcher stops the kernel and launches it
 * with the workgroups split in proportion (between 1/8 and 7/8).  It ends by itself after tens of
 * milliseconds without new tiles and is launched again when requests come;
 * aesgpu_server_destroy() stops it.  While it runs it holds every CU's LDS,
 * so other kernels on the device run only in the registers and waves it
 * leaves free (kernels that need LDS wait for it to end), and it holds the
 * hardware queue of its stream: work of other streams that the runtime maps
 * to the same hardware queue waits for it too.  n_streams, direct_requests
 * and the max_batch_* limits do not apply; at most 65,536 requests are in
 * flight, and stats.batches counts the kernel's launches.
 * Errors: EINVAL, EKEYLEN, ENOMEM, EHIP.
 */
int aesgpu_server_create(aesgpu_ctx *ctx, const uint8_t *keys, const uint16_t *key_bits,
                         size_t n_keys, const aesgpu_server_config *cfg, aesgpu_server **out);

/* Seconds since the server started (steady clock). */
double aesgpu_server_now(const aesgpu_server *server);

/*
 * Queues one request: ECB encrypt (dir 0) or decrypt (dir 1) of n_bytes (a
 * multiple of 16, at most the arena size) at device pointer d_in (16-byte
 * aligned, must stay valid until the request completes) with pool key key_id.
 * Requests are admitted first come first served as arena space frees up.
 * Returns EAGAIN when max_queued requests are already waiting; EINVAL /
 * EALIGN for bad arguments; a zero-length request completes at once.
 * Thread-safe.
 */
int aesgpu_server_submit(aesgpu_server *server, uint64_t req_id, int dir, uint32_t key_id,
                         const void *d_in, size_t n_bytes, double t_arrival);

/* Moves up to cap finished requests into out[]; *n_done receives the count. */
int aesgpu_server_poll(aesgpu_server *server, aesgpu_done *out, size_t cap, size_t *n_done);

/* Returns a finished request's output range (d_out, n_bytes) to the arena. */
int aesgpu_server_release(aesgpu_server *server, const void *d_out, size_t n_bytes);

int aesgpu_server_get_stats(aesgpu_server *server, aesgpu_server_stats *out);

/*
 * Load generator: submits reqs[i] at time t_start + reqs[i].t_arrival on the
 * server clock (in order, retrying while the queue is full), polls and
 * releases outputs as they finish, and returns when all n are done, with
 * done[req_id] filled.  Runs in the calling thread.  Errors: EINVAL, or the
 * first failed request's status.
 */
int aesgpu_server_replay(aesgpu_server *server, const aesgpu_request *reqs, size_t n,
                         double t_start, aesgpu_done *done);

/* Stops the dispatcher after the batches in flight finish and frees the
 * server (arena, schedules, streams).  NULL is ignored. */
void aesgpu_server_destroy(aesgpu_server *server);

/* Human-readable name of a status code (static string, never NULL). */
const char *aesgpu_strerror(int status);

/* Number of compute units the context launches for (host query only). */
int aesgpu_ctx_num_cus(const aesgpu_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* AESGPU_H */
