"""GPU parity at the full workload sizes (1 GiB per key size; 4 GiB CTR),
in the launch configuration the benchmark times.  The oracle recomputes
sampled blocks one by one (both ends, random positions, tile and grid-stride
edges); properties that hold at any size (decrypt(encrypt(x)) = x, CTR is its
own inverse) are checked on the whole buffer on the GPU."""
import numpy as np
import pytest

import oracle
from gpu_common import gather_blocks, log, requires_gpu, sample_indices, to_dev

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
def gib():
    from paper_1201_0398_amd import workloads
    log("generating 1 GiB workload (seed 1)")
    return workloads.single_1gib(seed=1)


@pytest.mark.parametrize("bits", [128, 192, 256])
def test_1gib_ecb(A, ctx, gib, bits):
    import torch
    log(f"case: 1 GiB ECB-{bits}")
    key = gib.keys[bits]
    k = A.aesgpu_expand_key(key)
    n = gib.data.size // 16
    d_in = to_dev(gib.data)
    d_ct = torch.empty_like(d_in)
    A.aesgpu_ecb_encrypt(ctx, k, d_in, d_ct)
    rng = np.random.default_rng(bits)
    idx = sample_indices(n, rng, boundaries=[TILE, GRID_STEP, n - GRID_STEP])
    got = gather_blocks(d_ct, idx)
    assert np.array_equal(got, oracle.ecb_sampled(key, gib.data, idx))
    d_pt = torch.empty_like(d_in)
    A.aesgpu_ecb_decrypt(ctx, k, d_ct, d_pt)
    assert torch.equal(d_pt, d_in), "decrypt(encrypt(x)) != x"
    A.aesgpu_ecb_decrypt(ctx, k, d_in, d_pt)
    got = gather_blocks(d_pt, idx)
    assert np.array_equal(got, oracle.ecb_sampled(key, gib.data, idx, decrypt=True))


def test_1gib_ctr128(A, ctx, gib):
    import torch
    log("case: 1 GiB CTR-128")
    key = gib.keys[128]
    k = A.aesgpu_expand_key(key)
    n = gib.data.size // 16
    d_in = to_dev(gib.data)
    d_out = torch.empty_like(d_in)
    A.aesgpu_ctr_xcrypt(ctx, k, gib.nonce, gib.ctr0, d_in, d_out)
    idx = sample_indices(n, np.random.default_rng(5), boundaries=[TILE, GRID_STEP])
    got = gather_blocks(d_out, idx)
    assert np.array_equal(got, oracle.ctr_sampled(key, gib.nonce, gib.ctr0, gib.data, idx))
    A.aesgpu_ctr_xcrypt(ctx, k, gib.nonce, gib.ctr0, d_out, d_out)
    assert torch.equal(d_out, d_in)


def test_4gib_ctr256(A, ctx):
    import torch
    from paper_1201_0398_amd import workloads
    log("case: 4 GiB CTR-256 seed 2 (generating)")
    w = workloads.ctr_4gib(seed=2)
    key = w.keys[256]
    k = A.aesgpu_expand_key(key)
    n = w.data.size // 16
    d_in = to_dev(w.data)
    d_out = torch.empty_like(d_in)
    A.aesgpu_ctr_xcrypt(ctx, k, w.nonce, w.ctr0, d_in, d_out)
    idx = sample_indices(n, np.random.default_rng(6), boundaries=[1 << 24, 1 << 27, GRID_STEP])
    got = gather_blocks(d_out, idx)
    assert np.array_equal(got, oracle.ctr_sampled(key, w.nonce, w.ctr0, w.data, idx))
    A.aesgpu_ctr_xcrypt(ctx, k, w.nonce, w.ctr0, d_out, d_out)
    assert torch.equal(d_out, d_in), "CTR(CTR(x)) != x over 4 GiB"
