"""Single-buffer calls that the library splits into several kernel launches.

A workgroup hands out its shares of work (16 per tile) from a 16-bit count in
LDS, so a call of more than 4095 tiles per CU is cut into parts of whole
tiles.  AESGPU_MAX_TILES_PER_CU (read at context creation) makes the parts
small enough to test here: at 2, a part is one tile per CU.  Every mode
against the oracle, with ragged ends, a CTR tail, a shifted CTR lane mapping,
an LE-128 counter whose word 0 wraps inside the call, and CBC chaining across
the part boundaries."""
import os

import numpy as np
import pytest

import oracle
from gpu_common import from_dev, log, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.fixture(scope="module", params=[1, 4], ids=["bpl1", "bpl4"])
def split(request):
    import torch
    from paper_1201_0398_amd import aesgpu as A
    env = {"AESGPU_FORCE_BPL": str(request.param), "AESGPU_MAX_TILES_PER_CU": "2"}
    old = {k: os.environ.pop(k, None) for k in env}
    os.environ.update(env)
    try:
        c = A.aesgpu_create()
    finally:
        for k, v in old.items():
            os.environ.pop(k, None)
            if v is not None:
                os.environ[k] = v
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    part = n_cu * 1024 * request.param        # blocks per launch: one tile per CU
    log(f"split context: {request.param} blocks per lane, {part} blocks per launch")
    yield A, c, part
    A.aesgpu_destroy(c)


def _sizes(part):
    # one part exactly, one block into a second part, two parts and a ragged third
    return [part, part + 1, 2 * part + 777]


def test_split_ecb(split):
    import torch
    A, ctx, part = split
    rng = np.random.default_rng(9100)
    key = rng.integers(0, 256, 16, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    for n in _sizes(part):
        log(f"case: split ECB-128 n_blocks={n}")
        data = rng.integers(0, 256, 16 * n, dtype=np.uint8)
        d_in = to_dev(data)
        d_ct, d_pt = torch.empty_like(d_in), torch.empty_like(d_in)
        A.aesgpu_ecb_encrypt(ctx, k, d_in, d_ct)
        A.aesgpu_ecb_decrypt(ctx, k, d_in, d_pt)
        assert np.array_equal(from_dev(d_ct), oracle.ecb_encrypt(key, data))
        assert np.array_equal(from_dev(d_pt), oracle.ecb_decrypt(key, data))


def test_split_ctr(split):
    import torch
    A, ctx, part = split
    rng = np.random.default_rng(9200)
    key = rng.integers(0, 256, 32, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    n_bytes = 16 * (2 * part + 777) + 9
    n_blocks = (n_bytes + 15) // 16
    for ctr0 in [0, (1 << 32) - n_blocks - 70]:     # the second shifts the lane mapping
        log(f"case: split CTR-256 n_bytes={n_bytes} ctr0={ctr0:#x}")
        nonce = rng.integers(0, 256, 12, dtype=np.uint8)
        data = rng.integers(0, 256, n_bytes, dtype=np.uint8)
        d_in = to_dev(data)
        d_out = torch.full((n_bytes + 64,), 0x5A, dtype=torch.uint8, device="cuda")
        A.aesgpu_ctr_xcrypt(ctx, k, nonce, ctr0, d_in, d_out, n_bytes)
        out = from_dev(d_out)
        assert np.array_equal(out[:n_bytes], oracle.ctr(key, nonce, ctr0, data))
        assert (out[n_bytes:] == 0x5A).all(), "wrote past the end"


def test_split_ctr_le128(split):
    import torch
    A, ctx, part = split
    rng = np.random.default_rng(9300)
    key = rng.integers(0, 256, 16, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    n_bytes = 16 * (2 * part + 777) + 5
    # word 0 of the counter wraps inside the second part
    iv = np.frombuffer((((1 << 32) - part - 100) | (0x0123456789ABCDEF << 32)).to_bytes(16, "little"),
                       dtype=np.uint8)
    for index0 in (0, 3):
        log(f"case: split CTR-LE128 n_bytes={n_bytes} index0={index0}")
        data = rng.integers(0, 256, n_bytes, dtype=np.uint8)
        d_in = to_dev(data)
        d_out = torch.empty_like(d_in)
        A.aesgpu_ctr_le128_xcrypt(ctx, k, iv, index0, d_in, d_out)
        assert np.array_equal(from_dev(d_out), oracle.ctr_le128(key, iv, index0, data))


@pytest.mark.parametrize("kb", [16, 32])
def test_split_cbc_decrypt(split, kb):
    import torch
    A, ctx, part = split
    rng = np.random.default_rng(9400 + kb)
    key = rng.integers(0, 256, kb, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    for n in _sizes(part):
        log(f"case: split CBC-{8 * kb} dec n_blocks={n}")
        iv = rng.integers(0, 256, 16, dtype=np.uint8)
        data = rng.integers(0, 256, 16 * n, dtype=np.uint8)
        d_in = to_dev(data)
        d_out = torch.empty_like(d_in)
        A.aesgpu_cbc_decrypt(ctx, k, iv, d_in, d_out)
        assert np.array_equal(from_dev(d_out), oracle.cbc_decrypt(key, iv, data))
