// Host runtime of the AES library: table construction, key expansion,
// argument validation and the C ABI entry points for single buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "aes_internal.h"

namespace aesgpu {
namespace {

// GF(2^8) with modulus x^8 + x^4 + x^3 + x + 1, by logarithms to the base 0x03
// (a generator of the multiplicative group).
struct Field {
    uint8_t exp[512];
    uint8_t log[256];

    Field() {
        uint8_t v = 1;
        for (int i = 0; i < 255; ++i) {
            exp[i] = v;
            exp[i + 255] = v;
            log[v] = static_cast<uint8_t>(i);
            // v *= 0x03, i.e. v ^ (v * 0x02)
            uint8_t dbl = static_cast<uint8_t>((v << 1) ^ ((v >> 7) * 0x1B));
            v = static_cast<uint8_t>(v ^ dbl);
        }
        exp[510] = exp[0];
        exp[511] = exp[1];
        log[0] = 0;
    }
    uint8_t mul(uint8_t a, uint8_t b) const {
        return (a && b) ? exp[log[a] + log[b]] : 0;
    }
    uint8_t inv(uint8_t a) const { return a ? exp[255 - log[a]] : 0; }
};

uint8_t rotl8(uint8_t v, int s) { return static_cast<uint8_t>((v << s) | (v >> (8 - s))); }
uint32_t rotl32(uint32_t v, int s) { return s ? (v << s) | (v >> (32 - s)) : v; }

HostTables build_tables() {
    const Field f;
    HostTables t{};
    for (int a = 0; a < 256; ++a) {
        // S(a) = b ^ (b<<<1) ^ (b<<<2) ^ (b<<<3) ^ (b<<<4) ^ 0x63, b = a^-1.
        const uint8_t b = f.inv(static_cast<uint8_t>(a));
        t.sbox[a] = static_cast<uint8_t>(b ^ rotl8(b, 1) ^ rotl8(b, 2) ^ rotl8(b, 3) ^
                                         rotl8(b, 4) ^ 0x63);
    }
    for (int a = 0; a < 256; ++a) t.inv_sbox[t.sbox[a]] = static_cast<uint8_t>(a);
    for (int x = 0; x < 256; ++x) {
        const uint8_t s = t.sbox[x];
        const uint8_t si = t.inv_sbox[x];
        // MixColumns column of (s,0,0,0): rows {2s, s, s, 3s}.
        const uint32_t te0 = uint32_t(f.mul(s, 2)) | (uint32_t(s) << 8) | (uint32_t(s) << 16) |
                             (uint32_t(f.mul(s, 3)) << 24);
        // InvMixColumns column of (si,0,0,0): rows {14si, 9si, 13si, 11si}.
        const uint32_t td0 = uint32_t(f.mul(si, 14)) | (uint32_t(f.mul(si, 9)) << 8) |
                             (uint32_t(f.mul(si, 13)) << 16) | (uint32_t(f.mul(si, 11)) << 24);
        for (int k = 0; k < 4; ++k) {
            // Row k instead of row 0 rotates the column down by k bytes.
            t.words[kTe + 256 * k + x] = rotl32(te0, 8 * k);
            t.words[kTd + 256 * k + x] = rotl32(td0, 8 * k);
        }
        t.words[kInvSS + x] = uint32_t(si) | (uint32_t(s) << 8);
    }
    return t;
}

uint32_t sub_word(uint32_t w, const uint8_t *sbox) {
    return uint32_t(sbox[w & 0xFF]) | (uint32_t(sbox[(w >> 8) & 0xFF]) << 8) |
           (uint32_t(sbox[(w >> 16) & 0xFF]) << 16) | (uint32_t(sbox[w >> 24]) << 24);
}

bool misaligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) != 0; }

// Partial overlap of [a, a+n) and [b, b+n); identical ranges are in place.
bool partial_overlap(const void *a, const void *b, uint64_t n) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    if (x == y || n == 0) return false;
    return x < y ? (y - x) < n : (x - y) < n;
}

// Common checks of a buffer call, in argument order.
int check_buffers(const aesgpu_ctx *ctx, const aesgpu_key *key, const void *in, const void *out,
                  uint64_t n_bytes, bool in_place_ok) {
    if (!ctx) return AESGPU_EINVAL;
    if (!key_ok(key)) return AESGPU_EINVAL;
    if (n_bytes == 0) return AESGPU_OK;
    if (!in || !out) return AESGPU_EINVAL;
    if (misaligned(in) || misaligned(out)) return AESGPU_EALIGN;
    if (in_place_ok ? partial_overlap(in, out, n_bytes)
                    : (partial_overlap(in, out, n_bytes) || in == out))
        return AESGPU_EINVAL;
    return AESGPU_OK;
}

// x (four little-endian words of a 128-bit integer) += v, modulo 2^128.
void add128(uint32_t (&x)[4], uint64_t v) {
    uint64_t carry = v;
    for (int c = 0; c < 4 && carry; ++c) {
        const uint64_t t = uint64_t(x[c]) + (carry & 0xFFFFFFFFull);
        x[c] = uint32_t(t);
        carry = (carry >> 32) + (t >> 32);
    }
}

// Round-1 constants of a counter block whose word `var` varies and whose other
// words are x[]: for output word c (Eq. (1) reads byte k of word (c + k) mod 4)
// the XOR of the round-1 key word and the three table terms that do not read
// word `var`.  x0 (the whitened fixed words) is passed through.
CtrConsts ctr_consts(const aesgpu_key *key, const uint32_t (&x)[4], int var, CtrConsts cc) {
    const HostTables &t = host_tables();
    uint32_t s[4];
    for (int c = 0; c < 4; ++c) s[c] = x[c] ^ key->enc[c];
    cc.kvar = key->enc[var];
    for (int c = 0; c < 4; ++c) {
        uint32_t p = key->enc[4 + c];
        for (int k = 0; k < 4; ++k) {
            const int i = (c + k) & 3;
            if (i == var) continue;
            p ^= t.words[kTe + 256 * k + ((s[i] >> (8 * k)) & 0xFF)];
        }
        cc.p[c] = p;
    }
    return cc;
}

int run(aesgpu_ctx *ctx, const LaunchArgs &a, aesgpu_stream_t stream) {
    DeviceGuard g(ctx->device);
    if (!g.ok()) return AESGPU_EHIP;
    LaunchArgs b = a;
    b.bpl = ctx->blocks_per_lane;
    b.max_tiles = ctx->max_tiles;
    return launch(ctx->d_tables, ctx->n_cu, b, reinterpret_cast<hipStream_t>(stream));
}

}  // namespace

bool key_ok(const aesgpu_key *k) {
    return k && ((k->key_bits == 128 && k->nr == 10) || (k->key_bits == 192 && k->nr == 12) ||
                 (k->key_bits == 256 && k->nr == 14));
}

const HostTables &host_tables() {
    static const HostTables t = build_tables();
    return t;
}

uint32_t inv_mix_column(uint32_t w) {
    // InvMixColumns(w) = sum_k Td_k[S(byte k of w)]: Td_k undoes the S-box
    // that S re-applies, leaving the InvMixColumns contribution of each row.
    const HostTables &t = host_tables();
    uint32_t r = 0;
    for (int k = 0; k < 4; ++k) r ^= t.words[kTd + 256 * k + t.sbox[(w >> (8 * k)) & 0xFF]];
    return r;
}

}  // namespace aesgpu

using namespace aesgpu;

extern "C" {

const char *aesgpu_strerror(int status) {
    switch (status) {
        case AESGPU_OK: return "ok";
        case AESGPU_EINVAL: return "invalid argument";
        case AESGPU_EKEYLEN: return "key length must be 16, 24 or 32 bytes";
        case AESGPU_EALIGN: return "device pointer not 16-byte aligned";
        case AESGPU_ECTR_OVERFLOW: return "32-bit block counter would wrap";
        case AESGPU_ENOMEM: return "out of memory";
        case AESGPU_EHIP: return "HIP runtime error";
        case AESGPU_EAGAIN: return "no free slot or memory; poll and retry";
        case AESGPU_ESCRATCH: return "batch larger than the allocation-free call's fixed scratch";
        default: return "unknown status";
    }
}

int aesgpu_expand_key(const uint8_t *key, size_t key_bytes, aesgpu_key *out) {
    if (!key || !out) return AESGPU_EINVAL;
    if (key_bytes != 16 && key_bytes != 24 && key_bytes != 32) return AESGPU_EKEYLEN;
    const HostTables &t = host_tables();
    const int nk = static_cast<int>(key_bytes / 4);
    const int nr = nk + 6;
    const int nw = 4 * (nr + 1);
    aesgpu_key k{};
    k.key_bits = static_cast<uint32_t>(32 * nk);
    k.nr = static_cast<uint32_t>(nr);
    for (int i = 0; i < nk; ++i) k.enc[i] = le32(key + 4 * i);
    uint8_t rcon = 1;
    for (int i = nk; i < nw; ++i) {
        uint32_t tmp = k.enc[i - 1];
        if (i % nk == 0) {
            // RotWord on the byte sequence is a right rotation of the LE word.
            tmp = sub_word((tmp >> 8) | (tmp << 24), t.sbox) ^ rcon;
            rcon = static_cast<uint8_t>((rcon << 1) ^ ((rcon >> 7) * 0x1B));
        } else if (nk == 8 && i % nk == 4) {
            tmp = sub_word(tmp, t.sbox);
        }
        k.enc[i] = k.enc[i - nk] ^ tmp;
    }
    for (int r = 0; r <= nr; ++r) {
        for (int c = 0; c < 4; ++c) {
            const uint32_t w = k.enc[4 * (nr - r) + c];
            k.dec[4 * r + c] = (r == 0 || r == nr) ? w : inv_mix_column(w);
        }
    }
    *out = k;
    return AESGPU_OK;
}

int aesgpu_create(aesgpu_ctx **out, int device) {
    if (!out) return AESGPU_EINVAL;
    *out = nullptr;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess) return AESGPU_EHIP;
    if (device < 0 || device >= n_dev) return AESGPU_EINVAL;
    DeviceGuard g(device);
    if (!g.ok()) return AESGPU_EHIP;
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        n_cu <= 0)
        return AESGPU_EHIP;
    // AESGPU_FORCE_BPL=1|2|4 fixes the single-buffer launches' blocks per lane
    // for this context (tests use it to run every kernel variant).
    int bpl = 0;
    if (const char *e = std::getenv("AESGPU_FORCE_BPL")) {
        const int v = std::atoi(e);
        if (v == 1 || v == 2 || v == 4) bpl = v;
    }
    // AESGPU_MAX_TILES_PER_CU=2..4096 splits single-buffer calls into launches
    // of fewer tiles (tests use it to cover the split on small buffers).
    uint32_t max_tiles = 0;
    if (const char *e = std::getenv("AESGPU_MAX_TILES_PER_CU")) {
        const long v = std::atol(e);
        if (v >= 2 && v <= long(kMaxTilesPerCu)) max_tiles = uint32_t(v);
    }
    aesgpu_ctx *ctx = new (std::nothrow) aesgpu_ctx{device, n_cu, nullptr, bpl, max_tiles};
    if (!ctx) return AESGPU_ENOMEM;
    const HostTables &t = host_tables();
    if (hipMalloc(&ctx->d_tables, sizeof(t.words)) != hipSuccess) {
        delete ctx;
        return AESGPU_ENOMEM;
    }
    if (hipMemcpy(ctx->d_tables, t.words, sizeof(t.words), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(ctx->d_tables);
        delete ctx;
        return AESGPU_EHIP;
    }
    *out = ctx;
    return AESGPU_OK;
}

void aesgpu_destroy(aesgpu_ctx *ctx) {
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        if (ctx->d_tables) (void)hipFree(ctx->d_tables);
    }
    delete ctx;
}

int aesgpu_ctx_num_cus(const aesgpu_ctx *ctx) { return ctx ? ctx->n_cu : AESGPU_EINVAL; }

static int ecb(aesgpu_ctx *ctx, const aesgpu_key *key, const void *in, void *out, size_t n_blocks,
               aesgpu_stream_t stream, bool decrypt) {
    if (n_blocks > (UINT64_MAX >> 4)) return AESGPU_EINVAL;
    const uint64_t n_bytes = uint64_t(n_blocks) * 16;
    int st = check_buffers(ctx, key, in, out, n_bytes, true);
    if (st != AESGPU_OK || n_bytes == 0) return st;
    LaunchArgs a{};
    a.op = decrypt ? Op::kEcbDec : Op::kEcbEnc;
    a.nr = key->nr;
    a.in = in;
    a.out = out;
    a.n_bytes = n_bytes;
    a.rk = reinterpret_cast<const RoundKeys *>(decrypt ? key->dec : key->enc);
    return run(ctx, a, stream);
}

int aesgpu_ecb_encrypt(aesgpu_ctx *ctx, const aesgpu_key *key, const void *d_in, void *d_out,
                       size_t n_blocks, aesgpu_stream_t stream) {
    return ecb(ctx, key, d_in, d_out, n_blocks, stream, false);
}

int aesgpu_ecb_decrypt(aesgpu_ctx *ctx, const aesgpu_key *key, const void *d_in, void *d_out,
                       size_t n_blocks, aesgpu_stream_t stream) {
    return ecb(ctx, key, d_in, d_out, n_blocks, stream, true);
}

int aesgpu_ctr_xcrypt(aesgpu_ctx *ctx, const aesgpu_key *key, const uint8_t *nonce, uint32_t ctr0,
                      const void *d_in, void *d_out, size_t n_bytes, aesgpu_stream_t stream) {
    if (!ctx || !key_ok(key) || !nonce) return AESGPU_EINVAL;
    int st = check_buffers(ctx, key, d_in, d_out, n_bytes, true);
    if (st != AESGPU_OK || n_bytes == 0) return st;
    const uint64_t n_blocks = (uint64_t(n_bytes) + 15) / 16;
    if (uint64_t(ctr0) + n_blocks - 1 > 0xFFFFFFFFull) return AESGPU_ECTR_OVERFLOW;
    LaunchArgs a{};
    a.op = Op::kCtrBe32;
    a.nr = key->nr;
    a.in = d_in;
    a.out = d_out;
    a.n_bytes = n_bytes;
    a.rk = reinterpret_cast<const RoundKeys *>(key->enc);
    a.ctr0 = ctr0;
    // Round-1 constants: counter words 0..2 are the nonce for every block.
    uint32_t x[4];
    for (int c = 0; c < 3; ++c) x[c] = le32(nonce + 4 * c);
    x[3] = 0;
    for (int c = 0; c < 3; ++c) a.ctr.x0[c] = x[c] ^ key->enc[c];
    a.ctr = ctr_consts(key, x, 3, a.ctr);
    return run(ctx, a, stream);
}

int aesgpu_ctr_le128_xcrypt(aesgpu_ctx *ctx, const aesgpu_key *key, const uint8_t *iv,
                            uint64_t index0, const void *d_in, void *d_out, size_t n_bytes,
                            aesgpu_stream_t stream) {
    if (!ctx || !key_ok(key) || !iv) return AESGPU_EINVAL;
    int st = check_buffers(ctx, key, d_in, d_out, n_bytes, true);
    if (st != AESGPU_OK || n_bytes == 0) return st;
    // Counter words 1..3 are folded into round-1 constants, so a launch must
    // not carry out of word 0: the call is split where word 0 wraps (at most
    // once per 2^32 blocks).
    const uint64_t n_blocks = (uint64_t(n_bytes) + 15) / 16;
    uint32_t x[4];
    for (int c = 0; c < 4; ++c) x[c] = le32(iv + 4 * c);
    add128(x, index0);
    for (uint64_t done = 0; done < n_blocks;) {
        const uint64_t room = (1ull << 32) - x[0];
        const uint64_t seg = std::min<uint64_t>(n_blocks - done, room);
        LaunchArgs a{};
        a.op = Op::kCtrLe128;
        a.nr = key->nr;
        a.in = static_cast<const uint8_t *>(d_in) + 16 * done;
        a.out = static_cast<uint8_t *>(d_out) + 16 * done;
        a.n_bytes = std::min<uint64_t>(16 * seg, uint64_t(n_bytes) - 16 * done);
        a.rk = reinterpret_cast<const RoundKeys *>(key->enc);
        for (int c = 0; c < 4; ++c) a.iv[c] = x[c];
        a.index0 = 0;
        a.ctr = ctr_consts(key, x, 0, a.ctr);
        st = run(ctx, a, stream);
        if (st != AESGPU_OK) return st;
        done += seg;
        add128(x, seg);
    }
    return AESGPU_OK;
}

int aesgpu_cbc_decrypt(aesgpu_ctx *ctx, const aesgpu_key *key, const uint8_t *iv,
                       const void *d_in, void *d_out, size_t n_blocks, aesgpu_stream_t stream) {
    if (!ctx || !key_ok(key) || !iv) return AESGPU_EINVAL;
    if (n_blocks > (UINT64_MAX >> 4)) return AESGPU_EINVAL;
    const uint64_t n_bytes = uint64_t(n_blocks) * 16;
    int st = check_buffers(ctx, key, d_in, d_out, n_bytes, false);
    if (st != AESGPU_OK || n_bytes == 0) return st;
    LaunchArgs a{};
    a.op = Op::kCbcDec;
    a.nr = key->nr;
    a.in = d_in;
    a.out = d_out;
    a.n_bytes = n_bytes;
    a.rk = reinterpret_cast<const RoundKeys *>(key->dec);
    for (int c = 0; c < 4; ++c) a.iv[c] = le32(iv + 4 * c);
    return run(ctx, a, stream);
}

}  // extern "C"
