"""GPU parity at the full workload sizes (1 GiB per key size; 4 GiB CTR), in
the launch configuration the benchmark times.  Every output byte is compared
with the oracle: the SHA-256 of the whole GPU output equals the digest of the
oracle's whole output (``golden/full_size_digests.json``, written by
``golden/make_full_digests.py`` from the oracle alone; the oracle takes about
half an hour over these workloads, so it is not re-run here).  The input's
digest is checked first, so a change in the input recipe shows as such.
CBC decryption runs on the 1 GiB buffer with the AES-128 and AES-256 keys, the
paper's LE-128 counter mode with the AES-192 key.
Sampled blocks are also recomputed by the oracle one by one (both ends,
random positions, tile and grid-stride edges), to name the first wrong block
if a digest differs."""
import numpy as np
import pytest

import oracle
from gpu_common import (full_size_digests, gather_blocks, log, requires_gpu, sample_indices,
                        sha256_dev, to_dev)

pytestmark = [pytest.mark.gpu, requires_gpu]

TILE = 4096
GRID_STEP = 256 * TILE


@pytest.fixture(scope="module")
def A():
    from paper_1201_0398_amd import aesgpu
    return aesgpu


@pytest.fixture(scope="module")
def ctx(A):
    c = A.aesgpu_create()
    yield c
    A.aesgpu_destroy(c)


@pytest.fixture(scope="module")
def digests():
    return full_size_digests()


@pytest.fixture(scope="module")
def gib(digests):
    import hashlib

    from paper_1201_0398_amd import workloads
    log("generating 1 GiB workload (seed 1)")
    w = workloads.single_1gib(seed=1)
    assert hashlib.sha256(memoryview(w.data)).hexdigest() == digests["gib1_input_sha256"], \
        "the 1 GiB input recipe changed"
    return w


@pytest.mark.parametrize("bits", [128, 192, 256])
def test_1gib_ecb(A, ctx, gib, digests, bits):
    import torch
    log(f"case: 1 GiB ECB-{bits}, whole buffer both ways")
    key = gib.keys[bits]
    k = A.aesgpu_expand_key(key)
    n = gib.data.size // 16
    d_in = to_dev(gib.data)
    d_ct = torch.empty_like(d_in)
    A.aesgpu_ecb_encrypt(ctx, k, d_in, d_ct)
    rng = np.random.default_rng(bits)
    idx = sample_indices(n, rng, boundaries=[TILE, GRID_STEP, n - GRID_STEP])
    assert np.array_equal(gather_blocks(d_ct, idx), oracle.ecb_sampled(key, gib.data, idx))
    assert sha256_dev(d_ct) == digests[f"gib1_ecb{bits}_encrypt_sha256"]
    d_pt = torch.empty_like(d_in)
    A.aesgpu_ecb_decrypt(ctx, k, d_ct, d_pt)
    assert torch.equal(d_pt, d_in), "decrypt(encrypt(x)) != x"
    A.aesgpu_ecb_decrypt(ctx, k, d_in, d_pt)
    assert np.array_equal(gather_blocks(d_pt, idx),
                          oracle.ecb_sampled(key, gib.data, idx, decrypt=True))
    assert sha256_dev(d_pt) == digests[f"gib1_ecb{bits}_decrypt_sha256"]


def test_1gib_ctr128(A, ctx, gib, digests):
    import torch
    log("case: 1 GiB CTR-128, whole buffer")
    key = gib.keys[128]
    k = A.aesgpu_expand_key(key)
    n = gib.data.size // 16
    d_in = to_dev(gib.data)
    d_out = torch.empty_like(d_in)
    A.aesgpu_ctr_xcrypt(ctx, k, gib.nonce, gib.ctr0, d_in, d_out)
    idx = sample_indices(n, np.random.default_rng(5), boundaries=[TILE, GRID_STEP])
    got = gather_blocks(d_out, idx)
    assert np.array_equal(got, oracle.ctr_sampled(key, gib.nonce, gib.ctr0, gib.data, idx))
    assert sha256_dev(d_out) == digests["gib1_ctr128_sha256"]
    A.aesgpu_ctr_xcrypt(ctx, k, gib.nonce, gib.ctr0, d_out, d_out)
    assert torch.equal(d_out, d_in)


@pytest.mark.parametrize("bits", [128, 256])
def test_1gib_cbc_decrypt(A, ctx, gib, digests, bits):
    """CBC decryption (Eq. (2)) of the whole 1 GiB buffer; IV = the
    workload's nonce then ctr0 as 4 big-endian bytes."""
    import torch
    log(f"case: 1 GiB CBC-{bits} decrypt, whole buffer")
    key = gib.keys[bits]
    k = A.aesgpu_expand_key(key)
    iv = np.concatenate([np.asarray(gib.nonce, dtype=np.uint8),
                         np.frombuffer(int(gib.ctr0).to_bytes(4, "big"), dtype=np.uint8)])
    n = gib.data.size // 16
    d_in = to_dev(gib.data)
    d_out = torch.empty_like(d_in)
    A.aesgpu_cbc_decrypt(ctx, k, iv, d_in, d_out)
    idx = sample_indices(n, np.random.default_rng(bits + 1), boundaries=[TILE, GRID_STEP])
    blocks = gib.data.reshape(n, 16)
    prev = np.where((idx == 0)[:, None], iv[None, :], blocks[np.maximum(idx, 1) - 1])
    want = oracle.ecb_sampled(key, gib.data, idx, decrypt=True) ^ prev
    assert np.array_equal(gather_blocks(d_out, idx), want)
    assert sha256_dev(d_out) == digests[f"gib1_cbc{bits}_decrypt_sha256"]


def test_1gib_ctr_le128_192(A, ctx, gib, digests):
    """The paper's LE-128 counter over the whole 1 GiB buffer, AES-192: IV
    word 0 = 2^32 - 2^25, so counter word 0 wraps halfway and the call is
    split there; words 1..3 = the workload's nonce."""
    import torch
    log("case: 1 GiB LE-128 CTR-192, whole buffer, word 0 wraps halfway")
    key = gib.keys[192]
    k = A.aesgpu_expand_key(key)
    iv = np.concatenate([np.frombuffer((2**32 - 2**25).to_bytes(4, "little"), dtype=np.uint8),
                         np.asarray(gib.nonce, dtype=np.uint8)])
    d_in = to_dev(gib.data)
    d_out = torch.empty_like(d_in)
    A.aesgpu_ctr_le128_xcrypt(ctx, k, iv, 0, d_in, d_out)
    n = gib.data.size // 16
    for lo in (0, (1 << 25) - 2048, n - 2048):
        want = oracle.ctr_le128(key, iv, lo, gib.data[16 * lo:16 * (lo + 4096)])
        assert np.array_equal(d_out[16 * lo:16 * (lo + 4096)].cpu().numpy(), want), f"blocks from {lo}"
    assert sha256_dev(d_out) == digests["gib1_ctrle128_192_sha256"]


def test_4gib_ctr256(A, ctx, digests):
    import hashlib

    import torch
    from paper_1201_0398_amd import workloads
    log("case: 4 GiB CTR-256 seed 2 (generating)")
    w = workloads.ctr_4gib(seed=2)
    assert hashlib.sha256(memoryview(w.data)).hexdigest() == digests["gib4_input_sha256"], \
        "the 4 GiB input recipe changed"
    key = w.keys[256]
    k = A.aesgpu_expand_key(key)
    n = w.data.size // 16
    d_in = to_dev(w.data)
    d_out = torch.empty_like(d_in)
    A.aesgpu_ctr_xcrypt(ctx, k, w.nonce, w.ctr0, d_in, d_out)
    idx = sample_indices(n, np.random.default_rng(6), boundaries=[1 << 24, 1 << 27, GRID_STEP])
    got = gather_blocks(d_out, idx)
    assert np.array_equal(got, oracle.ctr_sampled(key, w.nonce, w.ctr0, w.data, idx))
    assert sha256_dev(d_out) == digests["gib4_ctr256_sha256"], "4 GiB CTR-256 output"
    A.aesgpu_ctr_xcrypt(ctx, k, w.nonce, w.ctr0, d_out, d_out)
    assert torch.equal(d_out, d_in), "CTR(CTR(x)) != x over 4 GiB"
