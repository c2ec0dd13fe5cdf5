"""Seeded synthetic inputs for the AES workloads.

This module only draws random bytes and sizes; it holds none of the cipher's
arithmetic.  Both the GPU tests and the CPU oracle take their inputs from here,
so the two sides always see the same bytes.  Draw order is part of the recipe:
changing it changes every workload.

Workloads (all bytes uniform from ``numpy.random.default_rng(seed)``):

* ``single_small``  -- 1 MiB buffer, one AES-128 key (seed 0).
* ``single_1gib``   -- 1 GiB buffer, one key per key size (seed 1), plus a CTR
  nonce drawn after the buffer.
* ``ctr_4gib``      -- AES-256 key, 96-bit nonce, 4 GiB buffer (seed 2).
* ``batched``       -- messages of log-uniform length 16 B .. 1 MiB (16-byte
  multiples), each with its own key of uniform size and ECB or CTR (seed 3).
* ``serving``       -- a pool of keys of mixed size and a Poisson arrival trace
  of requests of log-uniform size 64 B .. 16 MiB, half encrypt half decrypt
  (seed 4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

KEY_BITS = (128, 192, 256)


def _bytes(rng: np.random.Generator, n: int) -> np.ndarray:
    return np.frombuffer(rng.bytes(n), dtype=np.uint8)


@dataclass
class SingleBuffer:
    keys: dict          # key_bits -> np.uint8 key
    data: np.ndarray    # uint8
    nonce: np.ndarray   # 12 bytes (CTR)
    ctr0: int
    iv: np.ndarray | None = None   # 16 bytes (CBC, LE-128 CTR), where drawn


def single_small(seed: int = 0, n_bytes: int = 1 << 20) -> SingleBuffer:
    """Key, data, nonce, then (drawn last, so the earlier draws are unchanged
    by it) a 16-byte IV for CBC and the LE-128 counter."""
    rng = np.random.default_rng(seed)
    key = _bytes(rng, 16)
    data = _bytes(rng, n_bytes)
    nonce = _bytes(rng, 12)
    iv = _bytes(rng, 16)
    return SingleBuffer({128: key}, data, nonce, 1, iv)


def single_1gib(seed: int = 1, n_bytes: int = 1 << 30) -> SingleBuffer:
    rng = np.random.default_rng(seed)
    keys = {bits: _bytes(rng, bits // 8) for bits in KEY_BITS}
    data = _bytes(rng, n_bytes)
    nonce = _bytes(rng, 12)
    return SingleBuffer(keys, data, nonce, 1)


def ctr_4gib(seed: int = 2, n_bytes: int = 1 << 32) -> SingleBuffer:
    rng = np.random.default_rng(seed)
    key = _bytes(rng, 32)
    nonce = _bytes(rng, 12)
    data = _bytes(rng, n_bytes)
    return SingleBuffer({256: key}, data, nonce, 1)


@dataclass
class Batch:
    lengths: np.ndarray     # bytes per message, int64
    offsets: np.ndarray     # byte offset of each message in the packed buffer
    key_bits: np.ndarray    # 128/192/256 per message
    keys: np.ndarray        # (m, 32) uint8, key bytes left-aligned, rest zero
    modes: np.ndarray       # 0 = ECB, 1 = CTR
    nonces: np.ndarray      # (m, 12) uint8 (zero for ECB messages)
    ctr0: np.ndarray        # uint32 per message
    data: np.ndarray        # packed input, uint8

    @property
    def total_bytes(self) -> int:
        return int(self.lengths.sum())


def log_uniform_lengths(rng: np.random.Generator, m: int, lo: int, hi: int) -> np.ndarray:
    """Lengths L = clamp(16*round(e^u / 16), lo, hi) with u ~ U(ln lo, ln hi)."""
    u = rng.uniform(math.log(lo), math.log(hi), size=m)
    L = 16 * np.rint(np.exp(u) / 16.0).astype(np.int64)
    return np.clip(L, lo, hi)


def batched(seed: int = 3, m: int = 65536, lo: int = 16, hi: int = 1 << 20) -> Batch:
    rng = np.random.default_rng(seed)
    lengths = log_uniform_lengths(rng, m, lo, hi)
    key_bits = np.asarray(KEY_BITS)[rng.integers(0, 3, size=m)]
    modes = rng.integers(0, 2, size=m).astype(np.uint8)
    keys = np.zeros((m, 32), dtype=np.uint8)
    nonces = np.zeros((m, 12), dtype=np.uint8)
    for j in range(m):
        nb = int(key_bits[j]) // 8
        keys[j, :nb] = _bytes(rng, nb)
        if modes[j] == 1:
            nonces[j] = _bytes(rng, 12)
    offsets = np.zeros(m, dtype=np.int64)
    if m > 1:
        offsets[1:] = np.cumsum(lengths)[:-1]
    data = _bytes(rng, int(lengths.sum()))
    return Batch(lengths, offsets, key_bits.astype(np.int64), keys, modes, nonces,
                 np.ones(m, dtype=np.uint32), data)


@dataclass
class CbcBatch:
    lengths: np.ndarray     # bytes per message (16-byte multiples)
    offsets: np.ndarray     # packed input offsets (outputs use the same)
    key_bits: np.ndarray
    keys: np.ndarray        # (m, 32) uint8, left-aligned
    ivs: np.ndarray         # (m, 16) uint8
    data: np.ndarray

    @property
    def total_bytes(self) -> int:
        return int(self.lengths.sum())


def cbc_batch(seed: int = 6, m: int = 65536, lo: int = 16, hi: int = 1 << 14) -> CbcBatch:
    """Many short CBC messages (the case where CBC encryption, sequential
    within a message, can use a GPU): log-uniform lengths, key size uniform
    over 128/192/256, per message a key then an IV, then the packed data."""
    rng = np.random.default_rng(seed)
    lengths = log_uniform_lengths(rng, m, lo, hi)
    key_bits = np.asarray(KEY_BITS)[rng.integers(0, 3, size=m)]
    keys = np.zeros((m, 32), dtype=np.uint8)
    ivs = np.zeros((m, 16), dtype=np.uint8)
    for j in range(m):
        nb = int(key_bits[j]) // 8
        keys[j, :nb] = _bytes(rng, nb)
        ivs[j] = _bytes(rng, 16)
    offsets = np.zeros(m, dtype=np.int64)
    if m > 1:
        offsets[1:] = np.cumsum(lengths)[:-1]
    data = _bytes(rng, int(lengths.sum()))
    return CbcBatch(lengths, offsets, key_bits.astype(np.int64), keys, ivs, data)


@dataclass
class ServingTrace:
    pool_bits: np.ndarray   # (n_keys,) 128/192/256
    pool_keys: np.ndarray   # (n_keys, 32) uint8, left-aligned
    arrivals: np.ndarray    # seconds from trace start, float64, nondecreasing
    sizes: np.ndarray       # request bytes (16-byte multiples)
    dirs: np.ndarray        # 0 = encrypt, 1 = decrypt
    key_ids: np.ndarray     # index into the pool
    src_offsets: np.ndarray  # byte offset of each request's input in the source pool
    source: np.ndarray      # device-resident random source bytes (uint8)


def serving(rate_per_s: float, n_requests: int, seed: int = 4, n_keys: int = 1024,
            lo: int = 64, hi: int = 1 << 24, source_bytes: int = 1 << 26) -> ServingTrace:
    """Key pool first, then the request trace, then the source pool.

    Each request's input is a 16-byte-aligned slice of ``source`` (which is
    kept smaller than the sum of requests so that it stays resident)."""
    rng = np.random.default_rng(seed)
    pool_bits = np.asarray(KEY_BITS)[rng.integers(0, 3, size=n_keys)].astype(np.int64)
    pool_keys = np.zeros((n_keys, 32), dtype=np.uint8)
    for j in range(n_keys):
        nb = int(pool_bits[j]) // 8
        pool_keys[j, :nb] = _bytes(rng, nb)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    arrivals = np.cumsum(gaps)
    sizes = log_uniform_lengths(rng, n_requests, lo, hi)
    dirs = rng.integers(0, 2, size=n_requests).astype(np.uint8)
    key_ids = rng.integers(0, n_keys, size=n_requests).astype(np.int64)
    source_bytes = max(int(source_bytes), int(hi))
    max_start = (source_bytes - sizes) // 16
    src_offsets = 16 * (rng.integers(0, 1 << 62, size=n_requests) % (max_start + 1))
    source = _bytes(rng, source_bytes)
    return ServingTrace(pool_bits, pool_keys, arrivals, sizes, dirs, key_ids,
                        src_offsets.astype(np.int64), source)
