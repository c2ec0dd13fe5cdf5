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
    AESGPU_EAGAIN = -7         /* server full: retry after polling */
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
 * *out receives the context.  Errors: EINVAL (out NULL, bad device), ENOMEM,
 * EHIP.
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

enum { AESGPU_MODE_ECB = 0, AESGPU_MODE_CTR = 1 };
enum { AESGPU_DIR_ENCRYPT = 0, AESGPU_DIR_DECRYPT = 1 };

/*
 * One message of a batch (host struct, 48 bytes).  Its input is
 * d_in + in_off and its output d_out + out_off (both 16-byte aligned), its key
 * the raw key bytes at d_keys + 32 * key_slot.  ECB messages are whole blocks
 * and use `dir`; CTR messages (nonce || BE32(ctr0 + i), as
 * aesgpu_ctr_xcrypt()) may end in a partial block and ignore `dir`.
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
 * 2048-block tiles).  tile_blocks must be a multiple of 64 * blocks_per_lane. */
typedef struct {
    uint32_t blocks_per_lane; /* 2 or 4 */
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
    uint32_t launches;         /* persistent launches per run (0, 1 or 2) */
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
 * KeyExpansion, plus the equivalent-inverse-cipher keys for ECB decryption).
 * d_keys holds n_key_slots raw keys at a 32-byte stride (key bytes first);
 * d_in and d_out are in_bytes / out_bytes long and must hold every message
 * (EINVAL otherwise).  d_in == d_out runs in place; other overlap is EINVAL.
 * Messages whose outputs overlap each other give undefined output.  By
 * default the launches are captured once into a hipGraph and replayed; the
 * graph is re-captured when d_keys, d_in or d_out change.  Calls on one plan
 * must not overlap in time (they share the plan's tile counters).
 * Errors: EINVAL, EALIGN, EHIP.
 */
int aesgpu_batch_run(aesgpu_batch *plan, const uint8_t *d_keys, size_t n_key_slots,
                     const void *d_in, size_t in_bytes, void *d_out, size_t out_bytes,
                     aesgpu_stream_t stream);

/* Plan statistics (host only).  Errors: EINVAL. */
int aesgpu_batch_info(const aesgpu_batch *plan, aesgpu_batch_stats *out);

/* Frees the plan (device descriptors, graph).  NULL is ignored.  The caller
 * must make sure no run of the plan is still executing. */
void aesgpu_batch_free(aesgpu_batch *plan);

/* Human-readable name of a status code (static string, never NULL). */
const char *aesgpu_strerror(int status);

/* Number of compute units the context launches for (host query only). */
int aesgpu_ctx_num_cus(const aesgpu_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* AESGPU_H */
