"""CPU oracle for AES block encryption -- test infrastructure only.

This package wraps ``aes_oracle.c``, a plain, literal C implementation of the
cipher that the paper (section 2.1) defers to FIPS-197 for, plus the paper's
T-table formulation (Eq. (1)) and the modes of section 3 (ECB, CTR, CBC
decryption per Eq. (2)).  Only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU library.

All buffers are numpy ``uint8`` arrays (or ``bytes``); keys are 16, 24 or 32
bytes.  Functions return new arrays and raise ``OracleError`` on a non-zero
status from the C side.

``Oracle(path)`` binds one compiled copy of the C file; the module-level
functions use the default copy ``oracle/_aes_oracle.so``.  The tests also build
deliberately broken copies (see ``build_variant``) to show that the pins catch
plausible mistakes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "aes_oracle.c")
_LIB = os.path.join(_HERE, "_aes_oracle.so")

OK = 0
EINVAL = -1
EKEYLEN = -2
ECTR_OVERFLOW = -4

_CFLAGS = ["-O2", "-std=c11", "-D_POSIX_C_SOURCE=200809L", "-Wall", "-Wextra", "-shared",
           "-fPIC", "-pthread"]


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


def _compile(src: str, out: str) -> None:
    tmp = out + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", *_CFLAGS, src, "-o", tmp])
    os.replace(tmp, out)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/_aes_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(SOURCE):
        _compile(SOURCE, _LIB)
    return _LIB


def build_variant(source_text: str, workdir: str, name: str) -> str:
    """Compile an edited copy of the oracle source (for the mutation tests)."""
    src = os.path.join(workdir, f"{name}.c")
    with open(src, "w") as f:
        f.write(source_text)
    out = os.path.join(workdir, f"{name}.so")
    _compile(src, out)
    return out


def _u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, memoryview)):
        a = np.frombuffer(bytes(a), dtype=np.uint8)
    return np.ascontiguousarray(a, dtype=np.uint8).reshape(-1)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _p64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _check(status: int, what: str) -> None:
    if status != OK:
        raise OracleError(status, what)


TRANSFORMS = {"sub_bytes": 0, "shift_rows": 1, "mix_columns": 2,
              "inv_sub_bytes": 3, "inv_shift_rows": 4, "inv_mix_columns": 5}


class Oracle:
    """One loaded copy of the C oracle."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        sz, ci, u8, u32, u64 = (ctypes.c_size_t, ctypes.c_int, ctypes.c_uint8, ctypes.c_uint32,
                                ctypes.c_uint64)
        sig = {
            "oracle_gf_mul": ([u8, u8], u8),
            "oracle_gf_inv": ([u8], u8),
            "oracle_sbox": ([u8], u8),
            "oracle_inv_sbox": ([u8], u8),
            "oracle_gf_mul_table": ([u8p], None),
            "oracle_transform": ([ci, u8p, u8p], ci),
            "oracle_key_expansion": ([u8p, ci, u8p], ci),
            "oracle_block": ([u8p, ci, ci, u8p, u8p], ci),
            "oracle_build_ttables": ([u32p, u32p], None),
            "oracle_ttable_ecb": ([u8p, ci, ci, u8p, u8p, sz], ci),
            "oracle_ttable_lookups_per_block": ([ci], ci),
            "oracle_ecb": ([u8p, ci, ci, u8p, u8p, sz, ci], ci),
            "oracle_ctr": ([u8p, ci, u8p, u32, u8p, u8p, sz, ci], ci),
            "oracle_ctr_le128": ([u8p, ci, u8p, u64, u8p, u8p, sz, ci], ci),
            "oracle_ctr_le128_blocks": ([u8p, u64, u8p, sz], None),
            "oracle_cbc_decrypt": ([u8p, ci, u8p, u8p, u8p, sz, ci], ci),
            "oracle_cbc_encrypt": ([u8p, ci, u8p, u8p, u8p, sz], ci),
            "oracle_ecb_sampled": ([u8p, ci, ci, u8p, u64p, sz, u8p], ci),
            "oracle_ctr_sampled": ([u8p, ci, u8p, u32, u8p, u64p, sz, u8p], ci),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        self.L = L
        self.path = path

    # ---- field and S-box ----------------------------------------------------

    def gf_mul(self, a: int, b: int) -> int:
        return int(self.L.oracle_gf_mul(a, b))

    def gf_inv(self, a: int) -> int:
        return int(self.L.oracle_gf_inv(a))

    def gf_mul_table(self) -> np.ndarray:
        """256x256 product table, [a, b] = a*b in GF(2^8)."""
        out = np.zeros(65536, dtype=np.uint8)
        self.L.oracle_gf_mul_table(_p(out))
        return out.reshape(256, 256)

    def sbox(self) -> np.ndarray:
        return np.array([self.L.oracle_sbox(a) for a in range(256)], dtype=np.uint8)

    def inv_sbox(self) -> np.ndarray:
        return np.array([self.L.oracle_inv_sbox(a) for a in range(256)], dtype=np.uint8)

    def transform(self, name: str, block) -> np.ndarray:
        """One state transform on a 16-byte block (state s[r][c] = in[r+4c])."""
        blk = _u8(block)
        assert blk.size == 16
        out = np.zeros(16, dtype=np.uint8)
        _check(self.L.oracle_transform(TRANSFORMS[name], _p(blk), _p(out)), name)
        return out

    def key_expansion(self, key) -> np.ndarray:
        """Schedule words as a (4*(Nr+1), 4) uint8 array, byte 0 first."""
        k = _u8(key)
        w = np.zeros(240, dtype=np.uint8)
        nr = self.L.oracle_key_expansion(_p(k), k.size, _p(w))
        if nr < 0:
            raise OracleError(nr, "key_expansion")
        return w[: 16 * (nr + 1)].reshape(-1, 4)

    def encrypt_block(self, key, block) -> np.ndarray:
        k, b = _u8(key), _u8(block)
        out = np.zeros(16, dtype=np.uint8)
        _check(self.L.oracle_block(_p(k), k.size, 0, _p(b), _p(out)), "encrypt_block")
        return out

    def decrypt_block(self, key, block) -> np.ndarray:
        k, b = _u8(key), _u8(block)
        out = np.zeros(16, dtype=np.uint8)
        _check(self.L.oracle_block(_p(k), k.size, 1, _p(b), _p(out)), "decrypt_block")
        return out

    # ---- the paper's T-table formulation ------------------------------------

    def ttables(self) -> tuple[np.ndarray, np.ndarray]:
        """(Te, Td) as (4, 256) uint32 arrays, little-endian columns."""
        te = np.zeros((4, 256), dtype=np.uint32)
        td = np.zeros((4, 256), dtype=np.uint32)
        self.L.oracle_build_ttables(te.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                    td.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        return te, td

    def ttable_ecb(self, key, data, decrypt: bool = False) -> np.ndarray:
        k, d = _u8(key), _u8(data)
        assert d.size % 16 == 0
        out = np.full_like(d, 0xA5)
        _check(self.L.oracle_ttable_ecb(_p(k), k.size, int(decrypt), _p(d), _p(out),
                                        d.size // 16), "ttable_ecb")
        return out

    def ttable_lookups_per_block(self, key_bytes: int) -> int:
        v = self.L.oracle_ttable_lookups_per_block(key_bytes)
        if v < 0:
            raise OracleError(v, "ttable_lookups_per_block")
        return int(v)

    # ---- modes --------------------------------------------------------------

    def ecb(self, key, data, decrypt: bool = False, threads: int = 0) -> np.ndarray:
        k, d = _u8(key), _u8(data)
        if d.size % 16:
            raise ValueError("ECB takes whole 16-byte blocks")
        out = np.full_like(d, 0xA5)
        _check(self.L.oracle_ecb(_p(k), k.size, int(decrypt), _p(d), _p(out), d.size // 16,
                                 threads), "ecb")
        return out

    def ecb_encrypt(self, key, data, threads: int = 0) -> np.ndarray:
        return self.ecb(key, data, False, threads)

    def ecb_decrypt(self, key, data, threads: int = 0) -> np.ndarray:
        return self.ecb(key, data, True, threads)

    def ctr(self, key, nonce, ctr0: int, data, threads: int = 0) -> np.ndarray:
        """CTR with nonce (12 bytes) || 32-bit big-endian counter from ctr0."""
        k, n, d = _u8(key), _u8(nonce), _u8(data)
        assert n.size == 12
        out = np.full_like(d, 0xA5)
        _check(self.L.oracle_ctr(_p(k), k.size, _p(n), ctr0, _p(d), _p(out), d.size, threads),
               "ctr")
        return out

    def ctr_le128(self, key, iv, index0: int, data, threads: int = 0) -> np.ndarray:
        """CTR with the paper's counter: IV + block index as a 128-bit LE integer."""
        k, v, d = _u8(key), _u8(iv), _u8(data)
        assert v.size == 16
        out = np.full_like(d, 0xA5)
        _check(self.L.oracle_ctr_le128(_p(k), k.size, _p(v), index0, _p(d), _p(out), d.size,
                                       threads), "ctr_le128")
        return out

    def ctr_le128_blocks(self, iv, index0: int, n_blocks: int) -> np.ndarray:
        v = _u8(iv)
        out = np.zeros(16 * n_blocks, dtype=np.uint8)
        self.L.oracle_ctr_le128_blocks(_p(v), index0, _p(out), n_blocks)
        return out

    def cbc_decrypt(self, key, iv, data, threads: int = 0) -> np.ndarray:
        k, v, d = _u8(key), _u8(iv), _u8(data)
        assert d.size % 16 == 0 and v.size == 16
        out = np.full_like(d, 0xA5)
        _check(self.L.oracle_cbc_decrypt(_p(k), k.size, _p(v), _p(d), _p(out), d.size // 16,
                                         threads), "cbc_decrypt")
        return out

    def cbc_encrypt(self, key, iv, data) -> np.ndarray:
        k, v, d = _u8(key), _u8(iv), _u8(data)
        assert d.size % 16 == 0 and v.size == 16
        out = np.full_like(d, 0xA5)
        _check(self.L.oracle_cbc_encrypt(_p(k), k.size, _p(v), _p(d), _p(out), d.size // 16),
               "cbc_encrypt")
        return out

    def ecb_sampled(self, key, data, idx, decrypt: bool = False) -> np.ndarray:
        """ECB of the blocks at indices ``idx`` only; returns (len(idx), 16)."""
        k, d = _u8(key), _u8(data)
        ix = np.ascontiguousarray(idx, dtype=np.uint64)
        if ix.size and int(ix.max()) >= d.size // 16:
            raise IndexError("block index out of range")
        out = np.zeros(16 * ix.size, dtype=np.uint8)
        _check(self.L.oracle_ecb_sampled(_p(k), k.size, int(decrypt), _p(d), _p64(ix), ix.size,
                                         _p(out)), "ecb_sampled")
        return out.reshape(-1, 16)

    def ctr_sampled(self, key, nonce, ctr0: int, data, idx) -> np.ndarray:
        """CTR output of the whole blocks at indices ``idx`` only; (len(idx), 16)."""
        k, n, d = _u8(key), _u8(nonce), _u8(data)
        ix = np.ascontiguousarray(idx, dtype=np.uint64)
        if ix.size and int(ix.max()) >= d.size // 16:
            raise IndexError("block index out of range")
        out = np.zeros(16 * ix.size, dtype=np.uint8)
        _check(self.L.oracle_ctr_sampled(_p(k), k.size, _p(n), ctr0, _p(d), _p64(ix), ix.size,
                                         _p(out)), "ctr_sampled")
        return out.reshape(-1, 16)


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def __getattr__(name):
    # Module-level access to the default copy: ``oracle.ecb_encrypt(...)``.
    if name.startswith("_"):
        raise AttributeError(name)
    return getattr(default(), name)
