/*
 * aes_oracle.c -- plain, slow, literal CPU reference for AES block encryption.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  The GPU library shares no code, header,
 * table or constant generator with it, and neither side includes the other.
 *
 * What it computes (paper, section 2.1): a block cipher over 128-bit blocks
 * with 128/192/256-bit keys and 10/12/14 rounds, each round made of SubBytes,
 * ShiftRows, MixColumns and AddRoundKey over GF(2^8) on a 4x4 byte state.  The
 * paper defers the definitions of those transforms, of the key schedule and of
 * the field to FIPS-197 (its reference [1]); this file writes those
 * definitions out byte by byte, in the order FIPS-197 applies them:
 *
 *   - GF(2^8) with modulus m(x) = x^8 + x^4 + x^3 + x + 1 (0x11B).
 *   - S-box = affine map (constant 0x63) of the multiplicative inverse,
 *     derived here at start-up, never typed in.  InvS = inverse permutation.
 *   - Cipher / InvCipher as the literal round sequences (FIPS-197 5.1, 5.3).
 *   - KeyExpansion (FIPS-197 5.2).
 *
 * It also holds the paper's own formulation (section 2.1, Eq. (1)): the state
 * as four 32-bit words and SubBytes+ShiftRows+MixColumns fused into four tables
 * T0..T3.  Those tables are built here from this file's S-box and MixColumns,
 * and the T-table cipher is checked against the literal cipher by the tests.
 *
 * Modes (paper, section 3): ECB and CTR encrypt/decrypt, CBC decrypt (Eq. (2))
 * and, for completeness of that check, sequential CBC encrypt.  The paper's own
 * CTR counter is a 128-bit little-endian add of the block index to the IV
 * (section 3, counter listing); the standard counter used by the library's
 * main CTR call is a 96-bit nonce followed by a 32-bit big-endian counter.
 *
 * Byte conventions: a block is the byte sequence in[0..15]; the state is
 * s[r][c] = in[r + 4c] (row r, column c).  A 32-bit word is little-endian over
 * four consecutive bytes, so word c of a block is column c and byte k of a word
 * is row k -- the paper's I_{c,k}.
 *
 * Threading: the mode functions split the block range into contiguous chunks
 * over POSIX threads.  Every block is still computed by the literal cipher;
 * threads only partition the loop.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_EKEYLEN (-2)
#define ORACLE_ECTR_OVERFLOW (-4)

/* ------------------------------------------------------------------------- */
/* GF(2^8)                                                                   */
/* ------------------------------------------------------------------------- */

/* Multiplication by x, reduced modulo m(x) = x^8 + x^4 + x^3 + x + 1. */
static uint8_t gf_xtime(uint8_t a)
{
    uint8_t shifted = (uint8_t)(a << 1);
    if (a & 0x80)
        shifted ^= 0x1B; /* x^8 = x^4 + x^3 + x + 1 (mod m) */
    return shifted;
}

/* Shift-and-add multiplication: a*b = sum over set bits i of b of a*x^i. */
uint8_t oracle_gf_mul(uint8_t a, uint8_t b)
{
    uint8_t acc = 0;
    while (b) {
        if (b & 1)
            acc ^= a;
        a = gf_xtime(a);
        b >>= 1;
    }
    return acc;
}

/* Multiplicative inverse a^254 (the group of nonzero elements has order 255),
 * by square-and-multiply.  By the FIPS-197 convention 0 maps to 0, which the
 * same power gives (0^254 = 0). */
uint8_t oracle_gf_inv(uint8_t a)
{
    uint8_t result = 1;
    uint8_t base = a;
    unsigned e = 254;
    while (e) {
        if (e & 1)
            result = oracle_gf_mul(result, base);
        base = oracle_gf_mul(base, base);
        e >>= 1;
    }
    return result;
}

/* Affine map over GF(2): bit i of the result is
 *   b_i ^ b_{i+4} ^ b_{i+5} ^ b_{i+6} ^ b_{i+7} ^ c_i   (indices mod 8),
 * with c = 0x63. */
static uint8_t affine_map(uint8_t b)
{
    uint8_t out = 0;
    for (int i = 0; i < 8; i++) {
        int bit = ((b >> i) ^ (b >> ((i + 4) & 7)) ^ (b >> ((i + 5) & 7)) ^
                   (b >> ((i + 6) & 7)) ^ (b >> ((i + 7) & 7)) ^ (0x63 >> i)) & 1;
        out |= (uint8_t)(bit << i);
    }
    return out;
}

static uint8_t SBOX[256];
static uint8_t INV_SBOX[256];
static pthread_once_t sbox_once = PTHREAD_ONCE_INIT;

static void derive_sboxes(void)
{
    for (int a = 0; a < 256; a++)
        SBOX[a] = affine_map(oracle_gf_inv((uint8_t)a));
    /* InvS is the inverse permutation, found by searching all 256 inputs. */
    for (int y = 0; y < 256; y++) {
        for (int x = 0; x < 256; x++) {
            if (SBOX[x] == y) {
                INV_SBOX[y] = (uint8_t)x;
                break;
            }
        }
    }
}

static void oracle_init(void) { pthread_once(&sbox_once, derive_sboxes); }

uint8_t oracle_sbox(uint8_t a)
{
    oracle_init();
    return SBOX[a];
}

uint8_t oracle_inv_sbox(uint8_t a)
{
    oracle_init();
    return INV_SBOX[a];
}

/* Full 256x256 product table (row a, column b), for the field checks. */
void oracle_gf_mul_table(uint8_t *out65536)
{
    for (int a = 0; a < 256; a++)
        for (int b = 0; b < 256; b++)
            out65536[a * 256 + b] = oracle_gf_mul((uint8_t)a, (uint8_t)b);
}

/* ------------------------------------------------------------------------- */
/* State transforms on s[r][c]                                               */
/* ------------------------------------------------------------------------- */

typedef uint8_t state_t[4][4]; /* [row][column] */

static void load_state(state_t s, const uint8_t in[16])
{
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            s[r][c] = in[r + 4 * c];
}

static void store_state(uint8_t out[16], state_t s)
{
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            out[r + 4 * c] = s[r][c];
}

static void sub_bytes(state_t s)
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = SBOX[s[r][c]];
}

static void inv_sub_bytes(state_t s)
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = INV_SBOX[s[r][c]];
}

/* Row r is rotated left by r positions: s'[r][c] = s[r][(c + r) mod 4]. */
static void shift_rows(state_t s)
{
    state_t t;
    memcpy(t, s, sizeof(t));
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = t[r][(c + r) % 4];
}

/* Row r is rotated right by r positions: s'[r][(c + r) mod 4] = s[r][c]. */
static void inv_shift_rows(state_t s)
{
    state_t t;
    memcpy(t, s, sizeof(t));
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][(c + r) % 4] = t[r][c];
}

/* Multiply every column by the circulant matrix whose first row is m[0..3]:
 * s'[r][c] = sum_k m[(k - r) mod 4] * s[k][c].  MixColumns uses the first row
 * {02, 03, 01, 01}; InvMixColumns uses {0E, 0B, 0D, 09}. */
static void circulant_columns(state_t s, const uint8_t m[4])
{
    for (int c = 0; c < 4; c++) {
        uint8_t col[4];
        for (int r = 0; r < 4; r++)
            col[r] = s[r][c];
        for (int r = 0; r < 4; r++) {
            uint8_t acc = 0;
            for (int k = 0; k < 4; k++)
                acc ^= oracle_gf_mul(m[(k - r + 4) % 4], col[k]);
            s[r][c] = acc;
        }
    }
}

static const uint8_t MIX_ROW[4] = {0x02, 0x03, 0x01, 0x01};
static const uint8_t INV_MIX_ROW[4] = {0x0E, 0x0B, 0x0D, 0x09};

static void mix_columns(state_t s) { circulant_columns(s, MIX_ROW); }
static void inv_mix_columns(state_t s) { circulant_columns(s, INV_MIX_ROW); }

/* Round key `round` is schedule words w[4*round .. 4*round+3]; word c is
 * XORed into column c, byte r of the word into row r. */
static void add_round_key(state_t s, const uint8_t w[][4], int round)
{
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            s[r][c] ^= w[4 * round + c][r];
}

/* Exported single-transform entry points on a 16-byte block, used by the
 * tests to check each transform by itself.  `which`: 0 SubBytes,
 * 1 ShiftRows, 2 MixColumns, 3 InvSubBytes, 4 InvShiftRows,
 * 5 InvMixColumns. */
int oracle_transform(int which, const uint8_t in[16], uint8_t out[16])
{
    oracle_init();
    state_t s;
    load_state(s, in);
    switch (which) {
    case 0: sub_bytes(s); break;
    case 1: shift_rows(s); break;
    case 2: mix_columns(s); break;
    case 3: inv_sub_bytes(s); break;
    case 4: inv_shift_rows(s); break;
    case 5: inv_mix_columns(s); break;
    default: return ORACLE_EINVAL;
    }
    store_state(out, s);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* KeyExpansion (FIPS-197 5.2)                                               */
/* ------------------------------------------------------------------------- */

/* Rcon[j] = (x^(j-1), 0, 0, 0), by repeated multiplication by x. */
static uint8_t rcon_byte(int j)
{
    uint8_t r = 0x01;
    for (int k = 1; k < j; k++)
        r = gf_xtime(r);
    return r;
}

/* Expands a 16/24/32-byte key into 4*(Nr+1) four-byte words w[i][0..3]
 * (byte 0 first, as FIPS-197 writes words).  Returns Nr, or ORACLE_EKEYLEN. */
int oracle_key_expansion(const uint8_t *key, int key_bytes, uint8_t w[60][4])
{
    oracle_init();
    if (key_bytes != 16 && key_bytes != 24 && key_bytes != 32)
        return ORACLE_EKEYLEN;
    const int nk = key_bytes / 4;
    const int nr = nk + 6;
    for (int i = 0; i < nk; i++)
        for (int b = 0; b < 4; b++)
            w[i][b] = key[4 * i + b];
    for (int i = nk; i < 4 * (nr + 1); i++) {
        uint8_t temp[4];
        memcpy(temp, w[i - 1], 4);
        if (i % nk == 0) {
            /* RotWord: [a0,a1,a2,a3] -> [a1,a2,a3,a0]; then SubWord; then Rcon. */
            uint8_t rot[4] = {temp[1], temp[2], temp[3], temp[0]};
            for (int b = 0; b < 4; b++)
                temp[b] = SBOX[rot[b]];
            temp[0] ^= rcon_byte(i / nk);
        } else if (nk > 6 && i % nk == 4) {
            for (int b = 0; b < 4; b++)
                temp[b] = SBOX[temp[b]];
        }
        for (int b = 0; b < 4; b++)
            w[i][b] = w[i - nk][b] ^ temp[b];
    }
    return nr;
}

/* ------------------------------------------------------------------------- */
/* Cipher / InvCipher (FIPS-197 5.1, 5.3), literal                           */
/* ------------------------------------------------------------------------- */

static void cipher(const uint8_t in[16], uint8_t out[16], const uint8_t w[][4], int nr)
{
    state_t s;
    load_state(s, in);
    add_round_key(s, w, 0);
    for (int round = 1; round < nr; round++) {
        sub_bytes(s);
        shift_rows(s);
        mix_columns(s);
        add_round_key(s, w, round);
    }
    sub_bytes(s);
    shift_rows(s);
    add_round_key(s, w, nr);
    store_state(out, s);
}

static void inv_cipher(const uint8_t in[16], uint8_t out[16], const uint8_t w[][4], int nr)
{
    state_t s;
    load_state(s, in);
    add_round_key(s, w, nr);
    for (int round = nr - 1; round >= 1; round--) {
        inv_shift_rows(s);
        inv_sub_bytes(s);
        add_round_key(s, w, round);
        inv_mix_columns(s);
    }
    inv_shift_rows(s);
    inv_sub_bytes(s);
    add_round_key(s, w, 0);
    store_state(out, s);
}

/* One block through the literal cipher (dir 0) or inverse cipher (dir 1). */
int oracle_block(const uint8_t *key, int key_bytes, int dir, const uint8_t in[16], uint8_t out[16])
{
    uint8_t w[60][4];
    int nr = oracle_key_expansion(key, key_bytes, w);
    if (nr < 0)
        return nr;
    if (dir == 0)
        cipher(in, out, w, nr);
    else if (dir == 1)
        inv_cipher(in, out, w, nr);
    else
        return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* The paper's T-table formulation (section 2.1, Eq. (1))                    */
/* ------------------------------------------------------------------------- */

/* Little-endian word over four bytes: byte k = row k. */
static uint32_t le_word(const uint8_t b[4])
{
    return (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
}

static uint8_t byte_of(uint32_t word, int k) { return (uint8_t)(word >> (8 * k)); }

/* T_k[x] is the column that MixColumns makes from a column holding S(x) in
 * row k and zero elsewhere (SubBytes and MixColumns fused, paper section 2.1).
 * Td_k[x] is the same with InvMixColumns and InvS, for the equivalent inverse
 * cipher.  Both are produced by running this file's own column transforms on
 * that one-hot column. */
void oracle_build_ttables(uint32_t te[4][256], uint32_t td[4][256])
{
    oracle_init();
    for (int k = 0; k < 4; k++) {
        for (int x = 0; x < 256; x++) {
            state_t s;
            memset(s, 0, sizeof(s));
            s[k][0] = SBOX[x];
            mix_columns(s);
            uint8_t col[4] = {s[0][0], s[1][0], s[2][0], s[3][0]};
            te[k][x] = le_word(col);

            memset(s, 0, sizeof(s));
            s[k][0] = INV_SBOX[x];
            inv_mix_columns(s);
            uint8_t dcol[4] = {s[0][0], s[1][0], s[2][0], s[3][0]};
            td[k][x] = le_word(dcol);
        }
    }
}

typedef struct {
    uint32_t te[4][256];
    uint32_t td[4][256];
} ttables_t;

static ttables_t TT;
static pthread_once_t tt_once = PTHREAD_ONCE_INIT;
static void build_tt(void) { oracle_build_ttables(TT.te, TT.td); }

/* Round keys as 32-bit words: K[round][c] = LE word w[4*round + c]. */
static void round_key_words(const uint8_t w[][4], int nr, uint32_t K[15][4])
{
    for (int round = 0; round <= nr; round++)
        for (int c = 0; c < 4; c++)
            K[round][c] = le_word(w[4 * round + c]);
}

/* Equivalent inverse cipher keys (FIPS-197 5.3.5): dk[0] = K[Nr],
 * dk[r] = InvMixColumns(K[Nr - r]) for 0 < r < Nr, dk[Nr] = K[0]. */
static void decrypt_key_words(const uint8_t w[][4], int nr, uint32_t DK[15][4])
{
    for (int round = 0; round <= nr; round++) {
        int src = nr - round;
        state_t s;
        for (int c = 0; c < 4; c++)
            for (int r = 0; r < 4; r++)
                s[r][c] = w[4 * src + c][r];
        if (round != 0 && round != nr)
            inv_mix_columns(s);
        for (int c = 0; c < 4; c++) {
            uint8_t col[4] = {s[0][c], s[1][c], s[2][c], s[3][c]};
            DK[round][c] = le_word(col);
        }
    }
}

/* Encryption with Eq. (1):
 *   O_c = T0[I_{c,0}] ^ T1[I_{c+1,1}] ^ T2[I_{c+2,2}] ^ T3[I_{c+3,3}] ^ K_c
 * (column indices mod 4) for the Nr-1 middle rounds, after an initial
 * AddRoundKey.  The last round has no MixColumns, so it substitutes through the
 * S-box with the same index pattern. */
static void ttable_encrypt(const uint8_t in[16], uint8_t out[16], const uint32_t K[15][4], int nr)
{
    uint32_t I[4], O[4];
    for (int c = 0; c < 4; c++)
        I[c] = le_word(in + 4 * c) ^ K[0][c];
    for (int round = 1; round < nr; round++) {
        for (int c = 0; c < 4; c++) {
            O[c] = TT.te[0][byte_of(I[c], 0)] ^ TT.te[1][byte_of(I[(c + 1) % 4], 1)] ^
                   TT.te[2][byte_of(I[(c + 2) % 4], 2)] ^ TT.te[3][byte_of(I[(c + 3) % 4], 3)] ^
                   K[round][c];
        }
        memcpy(I, O, sizeof(I));
    }
    for (int c = 0; c < 4; c++) {
        uint8_t col[4];
        for (int k = 0; k < 4; k++)
            col[k] = SBOX[byte_of(I[(c + k) % 4], k)];
        O[c] = le_word(col) ^ K[nr][c];
    }
    for (int c = 0; c < 4; c++)
        for (int k = 0; k < 4; k++)
            out[4 * c + k] = byte_of(O[c], k);
}

/* Decryption with the inverse tables; InvShiftRows turns the index pattern
 * into I_{c-k,k}. */
static void ttable_decrypt(const uint8_t in[16], uint8_t out[16], const uint32_t DK[15][4], int nr)
{
    uint32_t I[4], O[4];
    for (int c = 0; c < 4; c++)
        I[c] = le_word(in + 4 * c) ^ DK[0][c];
    for (int round = 1; round < nr; round++) {
        for (int c = 0; c < 4; c++) {
            O[c] = TT.td[0][byte_of(I[c], 0)] ^ TT.td[1][byte_of(I[(c + 3) % 4], 1)] ^
                   TT.td[2][byte_of(I[(c + 2) % 4], 2)] ^ TT.td[3][byte_of(I[(c + 1) % 4], 3)] ^
                   DK[round][c];
        }
        memcpy(I, O, sizeof(I));
    }
    for (int c = 0; c < 4; c++) {
        uint8_t col[4];
        for (int k = 0; k < 4; k++)
            col[k] = INV_SBOX[byte_of(I[(c + 4 - k) % 4], k)];
        O[c] = le_word(col) ^ DK[nr][c];
    }
    for (int c = 0; c < 4; c++)
        for (int k = 0; k < 4; k++)
            out[4 * c + k] = byte_of(O[c], k);
}

/* ECB over n blocks through the T-table formulation (single thread). */
int oracle_ttable_ecb(const uint8_t *key, int key_bytes, int dir, const uint8_t *in, uint8_t *out,
                      size_t n_blocks)
{
    pthread_once(&tt_once, build_tt);
    uint8_t w[60][4];
    int nr = oracle_key_expansion(key, key_bytes, w);
    if (nr < 0)
        return nr;
    uint32_t K[15][4];
    if (dir == 0)
        round_key_words(w, nr, K);
    else if (dir == 1)
        decrypt_key_words(w, nr, K);
    else
        return ORACLE_EINVAL;
    for (size_t i = 0; i < n_blocks; i++) {
        if (dir == 0)
            ttable_encrypt(in + 16 * i, out + 16 * i, K, nr);
        else
            ttable_decrypt(in + 16 * i, out + 16 * i, K, nr);
    }
    return ORACLE_OK;
}

/* Number of table reads the T-table formulation makes per block: 16 per
 * round for all Nr rounds (the last round reads the S-box with the same
 * pattern).  For a 128-bit key the paper counts 160 (section 2.1). */
int oracle_ttable_lookups_per_block(int key_bytes)
{
    if (key_bytes != 16 && key_bytes != 24 && key_bytes != 32)
        return ORACLE_EKEYLEN;
    return 16 * (key_bytes / 4 + 6);
}

/* ------------------------------------------------------------------------- */
/* Modes                                                                     */
/* ------------------------------------------------------------------------- */

/* The 16-byte counter block for block i of a CTR call with the standard
 * layout: nonce bytes 0..11, then ctr0 + i as a 32-bit big-endian integer. */
static void ctr_block_be32(const uint8_t nonce[12], uint32_t counter, uint8_t blk[16])
{
    memcpy(blk, nonce, 12);
    blk[12] = (uint8_t)(counter >> 24);
    blk[13] = (uint8_t)(counter >> 16);
    blk[14] = (uint8_t)(counter >> 8);
    blk[15] = (uint8_t)counter;
}

/* The paper's counter (section 3 listing): the IV read as a 128-bit
 * little-endian integer (32-bit word x least significant, then y, z, w) plus
 * the block index, modulo 2^128, written back little-endian.  The add is done
 * one byte at a time with an explicit carry. */
static void ctr_block_le128(const uint8_t iv[16], uint64_t index, uint8_t blk[16])
{
    unsigned carry = 0;
    for (int b = 0; b < 16; b++) {
        unsigned addend = (b < 8) ? (unsigned)((index >> (8 * b)) & 0xFF) : 0u;
        unsigned sum = (unsigned)iv[b] + addend + carry;
        blk[b] = (uint8_t)sum;
        carry = sum >> 8;
    }
}

enum { MODE_ECB = 0, MODE_CTR_BE32 = 1, MODE_CTR_LE128 = 2, MODE_CBC_DEC = 3 };

typedef struct {
    int mode;
    int dir;
    int nr;
    const uint8_t (*w)[4];
    const uint8_t *in;
    uint8_t *out;
    size_t n_bytes;     /* whole call; blocks are [0, ceil(n_bytes/16)) */
    size_t blk_begin;   /* this chunk's block range */
    size_t blk_end;
    const uint8_t *iv;  /* nonce (12 B) for CTR_BE32, IV (16 B) otherwise */
    uint32_t ctr0;
    uint64_t index0;
} job_t;

static void run_blocks(const job_t *j)
{
    for (size_t i = j->blk_begin; i < j->blk_end; i++) {
        const uint8_t *src = j->in + 16 * i;
        uint8_t *dst = j->out + 16 * i;
        if (j->mode == MODE_ECB) {
            if (j->dir == 0)
                cipher(src, dst, j->w, j->nr);
            else
                inv_cipher(src, dst, j->w, j->nr);
        } else if (j->mode == MODE_CBC_DEC) {
            /* Eq. (2): P_i = D_K(C_i) ^ C_{i-1}, with C_{-1} = IV. */
            uint8_t d[16];
            const uint8_t *prev = (i == 0) ? j->iv : j->in + 16 * (i - 1);
            inv_cipher(src, d, j->w, j->nr);
            for (int b = 0; b < 16; b++)
                dst[b] = d[b] ^ prev[b];
        } else {
            uint8_t ctr[16], ks[16];
            if (j->mode == MODE_CTR_BE32)
                ctr_block_be32(j->iv, (uint32_t)(j->ctr0 + i), ctr);
            else
                ctr_block_le128(j->iv, j->index0 + i, ctr);
            cipher(ctr, ks, j->w, j->nr);
            size_t len = j->n_bytes - 16 * i;
            if (len > 16)
                len = 16;
            for (size_t b = 0; b < len; b++)
                dst[b] = src[b] ^ ks[b];
        }
    }
}

static void *thread_main(void *arg)
{
    run_blocks((const job_t *)arg);
    return NULL;
}

/* Threads only partition the block range; a request for more than this is
   clamped to it (the job and thread arrays live on the stack). */
#define ORACLE_MAX_THREADS 512

static int resolve_threads(int threads, size_t n_blocks)
{
    if (threads <= 0) {
        long n = sysconf(_SC_NPROCESSORS_ONLN);
        threads = (n > 0) ? (int)n : 1;
    }
    if (threads > ORACLE_MAX_THREADS)
        threads = ORACLE_MAX_THREADS;
    if ((size_t)threads > n_blocks)
        threads = n_blocks ? (int)n_blocks : 1;
    return threads;
}

static int run_mode(const job_t *proto, size_t n_blocks, int threads)
{
    threads = resolve_threads(threads, n_blocks);
    if (threads == 1) {
        job_t j = *proto;
        j.blk_begin = 0;
        j.blk_end = n_blocks;
        run_blocks(&j);
        return ORACLE_OK;
    }
    pthread_t tid[ORACLE_MAX_THREADS];
    job_t jobs[ORACLE_MAX_THREADS];
    int started = 0;
    for (int t = 0; t < threads; t++) {
        jobs[t] = *proto;
        jobs[t].blk_begin = n_blocks * (size_t)t / (size_t)threads;
        jobs[t].blk_end = n_blocks * (size_t)(t + 1) / (size_t)threads;
        if (pthread_create(&tid[t], NULL, thread_main, &jobs[t]) != 0) {
            run_blocks(&jobs[t]); /* could not start a thread: do it here */
            tid[t] = 0;
        } else {
            started++;
        }
    }
    for (int t = 0; t < threads; t++)
        if (tid[t])
            pthread_join(tid[t], NULL);
    (void)started;
    return ORACLE_OK;
}

/* ECB encrypt (dir 0) or decrypt (dir 1) of n_blocks whole blocks. */
int oracle_ecb(const uint8_t *key, int key_bytes, int dir, const uint8_t *in, uint8_t *out,
               size_t n_blocks, int threads)
{
    uint8_t w[60][4];
    int nr = oracle_key_expansion(key, key_bytes, w);
    if (nr < 0)
        return nr;
    if (dir != 0 && dir != 1)
        return ORACLE_EINVAL;
    if (n_blocks == 0)
        return ORACLE_OK;
    job_t j = {MODE_ECB, dir, nr, (const uint8_t(*)[4])w, in, out, n_blocks * 16, 0, 0, NULL, 0, 0};
    return run_mode(&j, n_blocks, threads);
}

/* CTR with a 96-bit nonce and a 32-bit big-endian counter starting at ctr0.
 * Encryption and decryption are the same operation.  n_bytes need not be a
 * multiple of 16: the keystream of the last block is cut to length.  The
 * counter never wraps: ctr0 + ceil(n_bytes/16) - 1 must fit in 32 bits. */
int oracle_ctr(const uint8_t *key, int key_bytes, const uint8_t nonce[12], uint32_t ctr0,
               const uint8_t *in, uint8_t *out, size_t n_bytes, int threads)
{
    uint8_t w[60][4];
    int nr = oracle_key_expansion(key, key_bytes, w);
    if (nr < 0)
        return nr;
    size_t n_blocks = (n_bytes + 15) / 16;
    if (n_blocks == 0)
        return ORACLE_OK;
    if ((uint64_t)ctr0 + (uint64_t)n_blocks - 1 > 0xFFFFFFFFull)
        return ORACLE_ECTR_OVERFLOW;
    job_t j = {MODE_CTR_BE32, 0, nr, (const uint8_t(*)[4])w, in, out, n_bytes, 0, 0, nonce, ctr0, 0};
    return run_mode(&j, n_blocks, threads);
}

/* CTR with the paper's counter: block i uses IV + (index0 + i) as a 128-bit
 * little-endian integer, modulo 2^128. */
int oracle_ctr_le128(const uint8_t *key, int key_bytes, const uint8_t iv[16], uint64_t index0,
                     const uint8_t *in, uint8_t *out, size_t n_bytes, int threads)
{
    uint8_t w[60][4];
    int nr = oracle_key_expansion(key, key_bytes, w);
    if (nr < 0)
        return nr;
    size_t n_blocks = (n_bytes + 15) / 16;
    if (n_blocks == 0)
        return ORACLE_OK;
    job_t j = {MODE_CTR_LE128, 0, nr, (const uint8_t(*)[4])w, in, out, n_bytes, 0, 0, iv, 0, index0};
    return run_mode(&j, n_blocks, threads);
}

/* The counter blocks themselves for the paper's counter, for the tests. */
void oracle_ctr_le128_blocks(const uint8_t iv[16], uint64_t index0, uint8_t *out, size_t n_blocks)
{
    for (size_t i = 0; i < n_blocks; i++)
        ctr_block_le128(iv, index0 + i, out + 16 * i);
}

/* CBC decryption, Eq. (2): every block is decrypted independently and XORed
 * with the previous ciphertext block (the IV for the first). */
int oracle_cbc_decrypt(const uint8_t *key, int key_bytes, const uint8_t iv[16], const uint8_t *in,
                       uint8_t *out, size_t n_blocks, int threads)
{
    uint8_t w[60][4];
    int nr = oracle_key_expansion(key, key_bytes, w);
    if (nr < 0)
        return nr;
    if (n_blocks == 0)
        return ORACLE_OK;
    if (in == out)
        return ORACLE_EINVAL; /* needs the previous ciphertext block intact */
    job_t j = {MODE_CBC_DEC, 1, nr, (const uint8_t(*)[4])w, in, out, n_blocks * 16, 0, 0, iv, 0, 0};
    return run_mode(&j, n_blocks, threads);
}

/* CBC encryption: C_i = E_K(P_i ^ C_{i-1}), one block after the other. */
int oracle_cbc_encrypt(const uint8_t *key, int key_bytes, const uint8_t iv[16], const uint8_t *in,
                       uint8_t *out, size_t n_blocks)
{
    uint8_t w[60][4];
    int nr = oracle_key_expansion(key, key_bytes, w);
    if (nr < 0)
        return nr;
    uint8_t chain[16];
    memcpy(chain, iv, 16);
    for (size_t i = 0; i < n_blocks; i++) {
        uint8_t x[16];
        for (int b = 0; b < 16; b++)
            x[b] = in[16 * i + b] ^ chain[b];
        cipher(x, out + 16 * i, (const uint8_t(*)[4])w, nr);
        memcpy(chain, out + 16 * i, 16);
    }
    return ORACLE_OK;
}

/* ECB of selected blocks only: out[16*j..] = E/D(in[16*idx[j]..]).  Used to
 * check a large GPU output at sampled positions. */
int oracle_ecb_sampled(const uint8_t *key, int key_bytes, int dir, const uint8_t *in,
                       const uint64_t *idx, size_t n_idx, uint8_t *out)
{
    uint8_t w[60][4];
    int nr = oracle_key_expansion(key, key_bytes, w);
    if (nr < 0)
        return nr;
    for (size_t j = 0; j < n_idx; j++) {
        if (dir == 0)
            cipher(in + 16 * idx[j], out + 16 * j, (const uint8_t(*)[4])w, nr);
        else
            inv_cipher(in + 16 * idx[j], out + 16 * j, (const uint8_t(*)[4])w, nr);
    }
    return ORACLE_OK;
}

/* CTR (nonce || BE32 counter) keystream XOR data at selected whole blocks. */
int oracle_ctr_sampled(const uint8_t *key, int key_bytes, const uint8_t nonce[12], uint32_t ctr0,
                       const uint8_t *in, const uint64_t *idx, size_t n_idx, uint8_t *out)
{
    uint8_t w[60][4];
    int nr = oracle_key_expansion(key, key_bytes, w);
    if (nr < 0)
        return nr;
    for (size_t j = 0; j < n_idx; j++) {
        uint8_t ctr[16], ks[16];
        ctr_block_be32(nonce, (uint32_t)(ctr0 + idx[j]), ctr);
        cipher(ctr, ks, (const uint8_t(*)[4])w, nr);
        for (int b = 0; b < 16; b++)
            out[16 * j + b] = in[16 * idx[j] + b] ^ ks[b];
    }
    return ORACLE_OK;
}
