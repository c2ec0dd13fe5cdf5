"""Pins for the CPU oracle: checks against facts fixed outside the oracle.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises ``AssertionError``
when the oracle disagrees with the fact it checks.  The facts come from the
paper (Eq. (1)'s printed index pattern, the table-read count of section 2.1),
from the mathematics of GF(2^8) and of the cipher (field axioms, the order of
x under the AES modulus, inverse relations, the closed form of the MixColumns
polynomial inverse, the S-box's differential uniformity and nonlinearity), from
brute force on small cases, and from a black-box run of the system OpenSSL
(the only independent AES implementation available).  ``test_oracle_pins.py``
runs them on the oracle; ``test_oracle_mutants.py`` runs them on deliberately
broken copies and requires each copy to fail at least one.
"""
from __future__ import annotations

import os

import numpy as np

import openssl_ref

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
KEY_SIZES = (16, 24, 32)


def _read_eq1_pattern():
    """{c: [(i, k) for T_0..T_3]} from the paper's Eq. (1) fixture."""
    pattern = {}
    with open(os.path.join(GOLDEN, "eq1_index_pattern.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, *pairs = line.split()
            c = int(head.split("_")[1])
            pattern[c] = [tuple(int(v) for v in p.split(",")) for p in pairs]
    assert sorted(pattern) == [0, 1, 2, 3]
    return pattern


def _read_counts():
    out = {}
    with open(os.path.join(GOLDEN, "paper_counts.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = int(v)
    return out


def _words(block: np.ndarray) -> list[int]:
    return [int.from_bytes(bytes(block[4 * i:4 * i + 4]), "little") for i in range(4)]


def _block(words) -> np.ndarray:
    return np.frombuffer(b"".join(int(w).to_bytes(4, "little") for w in words), dtype=np.uint8)


# ---- GF(2^8) -----------------------------------------------------------------

def _clmul_mod(a: int, b: int, modulus: int = 0x11B) -> int:
    """Carry-less product of two bytes, then polynomial long division."""
    prod = 0
    for i in range(8):
        if (b >> i) & 1:
            prod ^= a << i
    for deg in range(14, 7, -1):
        if (prod >> deg) & 1:
            prod ^= modulus << (deg - 8)
    return prod


def pin_field(o, full: bool = True):
    T = o.gf_mul_table().astype(np.int64)
    a = np.arange(256)
    assert (T == T.T).all(), "multiplication not commutative"
    assert (T[1] == a).all() and (T[0] == 0).all(), "1 or 0 wrong"
    step = 1 if full else 17
    A, B, C = np.meshgrid(a[::step], a, a, indexing="ij")
    assert (T[A, B ^ C] == (T[A, B] ^ T[A, C])).all(), "not distributive over XOR"
    assert (T[T[A, B], C] == T[A, T[B, C]]).all(), "not associative"
    # Independent product: carry-less multiply and reduce modulo x^8+x^4+x^3+x+1.
    for x in range(0, 256, 1 if full else 7):
        for y in range(256):
            assert T[x, y] == _clmul_mod(x, y), f"{x:#x}*{y:#x}"


def pin_field_order(o):
    """Under x^8+x^4+x^3+x+1 the element x (0x02) has multiplicative order 51
    (the modulus is irreducible but not primitive) and 0x03 generates all 255
    nonzero elements."""
    T = o.gf_mul_table()

    def order(g):
        v, n = g, 1
        while v != 1:
            v = T[v, g]
            n += 1
            assert n <= 255, "element has no finite order: not a field"
        return n

    assert order(0x02) == 51
    assert order(0x03) == 255


def pin_inverse(o):
    T = o.gf_mul_table()
    assert o.gf_inv(0) == 0
    for a in range(1, 256):
        assert T[a, o.gf_inv(a)] == 1, f"inverse of {a:#x}"


# ---- S-box -------------------------------------------------------------------

def pin_sbox(o):
    S = o.sbox().astype(np.int64)
    Si = o.inv_sbox().astype(np.int64)
    a = np.arange(256)
    assert len(set(S.tolist())) == 256, "S-box not a permutation"
    assert S[0] == 0x63, "S(0) must be the affine constant (inverse of 0 is 0)"
    assert (S != a).all(), "S-box has a fixed point"
    assert (S != (a ^ 0xFF)).all(), "S-box has an opposite fixed point"
    assert (Si[S] == a).all() and (S[Si] == a).all(), "InvS is not the inverse"
    # S = affine(inverse): y -> S(inv(y)) ^ S(0) must be linear over GF(2).
    inv = np.array([o.gf_inv(int(v)) for v in a])
    L = S[inv] ^ S[0]
    Y1, Y2 = np.meshgrid(a, a, indexing="ij")
    assert (L[Y1 ^ Y2] == (L[Y1] ^ L[Y2])).all(), "S-box is not affine in the inverse"
    # Differential uniformity 4 and nonlinearity 112 (properties of inversion).
    du = 0
    for dx in range(1, 256):
        du = max(du, int(np.bincount(S ^ S[a ^ dx], minlength=256).max()))
    assert du == 4, f"differential uniformity {du}"
    pop = np.array([bin(v).count("1") & 1 for v in range(256)])
    PS = pop[np.bitwise_and.outer(a, S)]        # [b, x] = parity(b & S(x))
    PX = pop[np.bitwise_and.outer(a, a)]        # [c, x] = parity(c & x)
    W = (1 - 2 * PS) @ (1 - 2 * PX).T           # Walsh spectrum [b, c]
    assert 128 - np.abs(W[1:]).max() // 2 == 112, "nonlinearity"


# ---- ShiftRows / MixColumns ----------------------------------------------------

def pin_shift_rows_eq1(o):
    """ShiftRows moves byte k of word (i) to column c exactly as the paper's
    Eq. (1) prints: output word c takes I_{i,k} for the listed (i, k)."""
    pattern = _read_eq1_pattern()
    labels = np.arange(16, dtype=np.uint8)      # byte k of word i has label 4i+k
    out = o.transform("shift_rows", labels)
    for c in range(4):
        for k, (i, kk) in enumerate(pattern[c]):
            assert kk == k
            assert out[4 * c + k] == 4 * i + k, f"O_{c} byte {k}"
    back = o.transform("inv_shift_rows", out)
    assert (back == labels).all(), "InvShiftRows does not undo ShiftRows"


def _poly_mul_mod_x4_1(T, p, q):
    """Product of two polynomials over GF(2^8) (coefficient lists, degree <= 3)
    modulo x^4 + 1, i.e. with exponents taken mod 4."""
    r = [0, 0, 0, 0]
    for i in range(4):
        for j in range(4):
            r[(i + j) % 4] ^= int(T[p[i], q[j]])
    return r


def pin_mix_columns(o, n_random: int = 2000, seed: int = 11):
    T = o.gf_mul_table()
    e0 = np.zeros(16, dtype=np.uint8)
    e0[0] = 1
    # Column 0 of the MixColumns matrix is the product of the column polynomial
    # by x^0, i.e. the coefficients of c(x) (row r holds coefficient of x^r).
    c = [int(v) for v in o.transform("mix_columns", e0)[:4]]
    d = [int(v) for v in o.transform("inv_mix_columns", e0)[:4]]
    assert _poly_mul_mod_x4_1(T, c, d) == [1, 0, 0, 0], "c(x)*d(x) != 1 mod x^4+1"
    rng = np.random.default_rng(seed)
    for _ in range(n_random):
        a = rng.integers(0, 256, 16, dtype=np.uint8)
        b = rng.integers(0, 256, 16, dtype=np.uint8)
        ma = o.transform("mix_columns", a)
        assert (o.transform("inv_mix_columns", ma) == a).all()
        assert (o.transform("mix_columns", a ^ b) == (ma ^ o.transform("mix_columns", b))).all()
    for pos in range(4):
        for v in range(256):
            col = np.zeros(16, dtype=np.uint8)
            col[pos] = v
            assert (o.transform("inv_mix_columns", o.transform("mix_columns", col)) == col).all()


# ---- Eq. (1) and the cipher ------------------------------------------------------

def pin_eq1_round(o, n: int = 500, seed: int = 12):
    """One middle round written as the paper's Eq. (1), with the index pattern
    read from the fixture and the oracle's T-tables, equals SubBytes,
    ShiftRows, MixColumns and AddRoundKey applied one after the other; the
    decryption tables do the same for the inverse transforms."""
    te, td = o.ttables()
    pattern = _read_eq1_pattern()
    rng = np.random.default_rng(seed)
    for _ in range(n):
        blk = rng.integers(0, 256, 16, dtype=np.uint8)
        key = rng.integers(0, 256, 16, dtype=np.uint8)
        I, K = _words(blk), _words(key)
        O = []
        for c in range(4):
            v = K[c]
            for t, (i, k) in enumerate(pattern[c]):
                v ^= int(te[t][(I[i] >> (8 * k)) & 0xFF])
            O.append(v)
        ref = o.transform("mix_columns", o.transform("shift_rows", o.transform("sub_bytes", blk)))
        assert (_block(O) == (ref ^ key)).all(), "Eq. (1) round"
        # Inverse round of the equivalent inverse cipher: InvShiftRows turns
        # the pattern's word index i = c+k into c-k.
        Od = []
        for c in range(4):
            v = K[c]
            for t in range(4):
                v ^= int(td[t][(I[(c - t) % 4] >> (8 * t)) & 0xFF])
            Od.append(v)
        refd = o.transform("inv_mix_columns",
                           o.transform("inv_shift_rows", o.transform("inv_sub_bytes", blk)))
        assert (_block(Od) == (refd ^ key)).all(), "inverse T-table round"


def pin_lookup_count(o):
    counts = _read_counts()
    assert o.ttable_lookups_per_block(16) == counts["aes128_lookups_per_block"]
    assert counts["round_lookups"] * counts["aes128_rounds"] == counts["aes128_lookups_per_block"]


def pin_ttable_cipher(o, n_blocks: int = 10000, seed: int = 13):
    rng = np.random.default_rng(seed)
    for kb in KEY_SIZES:
        key = rng.integers(0, 256, kb, dtype=np.uint8)
        data = rng.integers(0, 256, 16 * n_blocks, dtype=np.uint8)
        enc = o.ecb_encrypt(key, data)
        assert (o.ttable_ecb(key, data) == enc).all(), f"T-table encrypt, {kb * 8}-bit key"
        assert (o.ttable_ecb(key, data, decrypt=True) == o.ecb_decrypt(key, data)).all(), \
            f"T-table decrypt, {kb * 8}-bit key"


def pin_round_trip(o, n_blocks: int = 4096, seed: int = 14):
    rng = np.random.default_rng(seed)
    for kb in KEY_SIZES:
        key = rng.integers(0, 256, kb, dtype=np.uint8)
        data = rng.integers(0, 256, 16 * n_blocks, dtype=np.uint8)
        enc = o.ecb_encrypt(key, data)
        assert not (enc == data).all()
        assert (o.ecb_decrypt(key, enc) == data).all(), f"round trip, {kb * 8}-bit key"


def pin_key_schedule_prefix(o, seed: int = 15):
    rng = np.random.default_rng(seed)
    for kb in KEY_SIZES:
        key = rng.integers(0, 256, kb, dtype=np.uint8)
        w = o.key_expansion(key)
        assert w.shape == (4 * (kb // 4 + 7), 4)
        assert (w[: kb // 4].reshape(-1) == key).all()


# ---- OpenSSL black box -------------------------------------------------------------

def pin_openssl(o, n_blocks: int = 64, seed: int = 16):
    """ECB both ways, CTR and CBC decryption agree with the system OpenSSL for
    random keys of all three sizes."""
    rng = np.random.default_rng(seed)
    for kb in KEY_SIZES:
        bits = 8 * kb
        for _ in range(3):
            key = rng.integers(0, 256, kb, dtype=np.uint8)
            data = rng.integers(0, 256, 16 * n_blocks, dtype=np.uint8)
            ref = openssl_ref.enc(f"aes-{bits}-ecb", bytes(key), bytes(data))
            assert bytes(o.ecb_encrypt(key, data)) == ref, f"ECB-{bits} encrypt vs OpenSSL"
            ref_d = openssl_ref.enc(f"aes-{bits}-ecb", bytes(key), bytes(data), decrypt=True)
            assert bytes(o.ecb_decrypt(key, data)) == ref_d, f"ECB-{bits} decrypt vs OpenSSL"
            nonce = rng.integers(0, 256, 12, dtype=np.uint8)
            ctr0 = int(rng.integers(0, 1 << 31))
            tail = 16 * n_blocks - int(rng.integers(0, 16))
            iv = bytes(nonce) + ctr0.to_bytes(4, "big")
            ref_c = openssl_ref.enc(f"aes-{bits}-ctr", bytes(key), bytes(data[:tail]), iv=iv,
                                    nopad=False)
            assert bytes(o.ctr(key, nonce, ctr0, data[:tail])) == ref_c, f"CTR-{bits} vs OpenSSL"
            civ = rng.integers(0, 256, 16, dtype=np.uint8)
            ref_b = openssl_ref.enc(f"aes-{bits}-cbc", bytes(key), bytes(data), iv=bytes(civ),
                                    decrypt=True)
            assert bytes(o.cbc_decrypt(key, civ, data)) == ref_b, f"CBC-{bits} decrypt vs OpenSSL"
            ref_be = openssl_ref.enc(f"aes-{bits}-cbc", bytes(key), bytes(data), iv=bytes(civ))
            assert bytes(o.cbc_encrypt(key, civ, data)) == ref_be, f"CBC-{bits} encrypt vs OpenSSL"


# ---- modes -------------------------------------------------------------------------

def pin_ctr_properties(o, seed: int = 17):
    rng = np.random.default_rng(seed)
    key = rng.integers(0, 256, 32, dtype=np.uint8)
    nonce = rng.integers(0, 256, 12, dtype=np.uint8)
    data = rng.integers(0, 256, 16 * 300 + 9, dtype=np.uint8)
    ct = o.ctr(key, nonce, 1, data)
    assert (o.ctr(key, nonce, 1, ct) == data).all(), "CTR is not an involution"
    # Keystream is the cipher of the counter blocks.
    ks = ct ^ data
    ctr_blocks = np.frombuffer(b"".join(bytes(nonce) + (1 + i).to_bytes(4, "big")
                                        for i in range(301)), dtype=np.uint8)
    assert (o.ecb_encrypt(key, ctr_blocks)[: data.size] == ks).all(), "CTR keystream"
    # Chunks that advance the counter equal one call.
    cut = 16 * 77
    parts = np.concatenate([o.ctr(key, nonce, 1, data[:cut]),
                            o.ctr(key, nonce, 1 + 77, data[cut:])])
    assert (parts == ct).all(), "chunked CTR"
    # Tail truncation: a shorter message is a prefix.
    assert (o.ctr(key, nonce, 1, data[:37]) == ct[:37]).all()
    # The counter never wraps.
    try:
        o.ctr(key, nonce, 0xFFFFFFFF, data[:32])
    except Exception as e:  # noqa: BLE001
        assert getattr(e, "status", None) == -4
    else:
        raise AssertionError("CTR wrap not rejected")
    assert o.ctr(key, nonce, 0xFFFFFFFF, data[:16]).size == 16


def pin_ctr_le128(o, seed: int = 18):
    """The paper's counter (section 3 listing) is the IV plus the block index as
    a 128-bit little-endian integer; checked against Python integers, across
    every word carry and the 2^128 wrap."""
    rng = np.random.default_rng(seed)
    ivs = [rng.integers(0, 256, 16, dtype=np.uint8) for _ in range(4)]
    ivs.append(np.frombuffer((0xFFFFFFFF).to_bytes(4, "little") + bytes(12), dtype=np.uint8))
    ivs.append(np.frombuffer(((1 << 96) - 3).to_bytes(16, "little"), dtype=np.uint8))
    ivs.append(np.frombuffer(((1 << 128) - 2).to_bytes(16, "little"), dtype=np.uint8))
    for iv in ivs:
        base = int.from_bytes(bytes(iv), "little")
        for index0 in (0, 5, (1 << 32) - 3):
            got = o.ctr_le128_blocks(iv, index0, 8)
            want = b"".join(((base + index0 + i) % (1 << 128)).to_bytes(16, "little")
                            for i in range(8))
            assert bytes(got) == want, "LE-128 counter"
    key = rng.integers(0, 256, 16, dtype=np.uint8)
    data = rng.integers(0, 256, 16 * 9 + 5, dtype=np.uint8)
    ctrs = o.ctr_le128_blocks(ivs[-1], 0, 10)
    ks = o.ecb_encrypt(key, ctrs)[: data.size]
    assert (o.ctr_le128(key, ivs[-1], 0, data) == (data ^ ks)).all(), "LE-128 CTR keystream"


def pin_cbc(o, seed: int = 19):
    rng = np.random.default_rng(seed)
    for kb in KEY_SIZES:
        key = rng.integers(0, 256, kb, dtype=np.uint8)
        iv = rng.integers(0, 256, 16, dtype=np.uint8)
        data = rng.integers(0, 256, 16 * 200, dtype=np.uint8)
        ct = o.cbc_encrypt(key, iv, data)
        assert (o.cbc_decrypt(key, iv, ct) == data).all(), "CBC round trip"
        assert (o.cbc_decrypt(key, iv, ct, threads=1) == data).all()


def pin_sampled(o, seed: int = 20):
    rng = np.random.default_rng(seed)
    key = rng.integers(0, 256, 24, dtype=np.uint8)
    data = rng.integers(0, 256, 16 * 500, dtype=np.uint8)
    idx = rng.integers(0, 500, 50)
    for dec in (False, True):
        full = o.ecb(key, data, dec).reshape(-1, 16)
        assert (o.ecb_sampled(key, data, idx, dec) == full[idx]).all()
    nonce = rng.integers(0, 256, 12, dtype=np.uint8)
    full = o.ctr(key, nonce, 9, data).reshape(-1, 16)
    assert (o.ctr_sampled(key, nonce, 9, data, idx) == full[idx]).all()


def pin_threads(o, seed: int = 21):
    rng = np.random.default_rng(seed)
    key = rng.integers(0, 256, 16, dtype=np.uint8)
    data = rng.integers(0, 256, 16 * 1001, dtype=np.uint8)
    a = o.ecb_encrypt(key, data, threads=1)
    for t in (2, 3, 7, 0):
        assert (o.ecb_encrypt(key, data, threads=t) == a).all()


ALL_PINS = [pin_field, pin_field_order, pin_inverse, pin_sbox, pin_shift_rows_eq1,
            pin_mix_columns, pin_eq1_round, pin_lookup_count, pin_ttable_cipher, pin_round_trip,
            pin_key_schedule_prefix, pin_openssl, pin_ctr_properties, pin_ctr_le128, pin_cbc,
            pin_sampled, pin_threads]
