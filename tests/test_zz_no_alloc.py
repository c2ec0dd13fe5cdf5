"""GPU test of aesgpu_batch_run_noalloc(), the batch call that allocates no
device memory (its descriptors go to a fixed per-GPU scratch area): its
output equals aesgpu_batch_run()'s on the same batch, bit for bit, on two
calls in a row (the second batch smaller, so stale scratch contents from the
first would show), bytes outside the messages' outputs stay untouched, and a
batch larger than the scratch is refused before any HIP call."""
import numpy as np
import pytest

from gpu_common import from_dev, log, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]


@pytest.fixture(scope="module")
def A():
    from paper_1201_0398_amd import aesgpu
    return aesgpu


@pytest.fixture(scope="module")
def ctx(A):
    c = A.aesgpu_create()
    yield c
    A.aesgpu_destroy(c)


def _batch(A, rng, m, max_blocks):
    """Mixed batch: ECB, CTR (ragged tails) and CBC messages, both
    directions, all key sizes, packed with gaps; outputs in reverse order."""
    modes = rng.integers(0, 3, size=m)
    lengths = 16 * rng.integers(1, max_blocks + 1, size=m)
    lengths = np.where(modes == 1, np.maximum(lengths - rng.integers(0, 16, size=m), 1), lengths)
    bits = np.array([128, 192, 256])[rng.integers(0, 3, size=m)]
    dirs = rng.integers(0, 2, size=m)
    span = 16 * ((lengths + 15) // 16) + 16 * rng.integers(0, 3, size=m)
    in_off = np.concatenate([[0], np.cumsum(span)[:-1]])
    out_off = np.concatenate([[0], np.cumsum(span[::-1])[:-1]])[::-1].copy()
    keys = rng.integers(0, 256, (m, 32), dtype=np.uint8)
    nonces = rng.integers(0, 256, (m, 12), dtype=np.uint8)
    ivs = rng.integers(0, 256, (m, 16), dtype=np.uint8)
    ctr0 = rng.integers(0, 1 << 31, size=m).astype(np.uint32)
    msgs = A.make_msgs(in_off, out_off, lengths, np.arange(m), bits, modes, dirs, nonces, ctr0,
                       iv=ivs)
    total = int(span.sum())
    return msgs, keys, rng.integers(0, 256, total, dtype=np.uint8), total


def _planned(A, ctx, msgs, d_keys, m, d_in, total, bpl, tile):
    import torch
    d_out = torch.full((total,), 0x5A, dtype=torch.uint8, device="cuda")
    plan = A.aesgpu_batch_plan(ctx, msgs, blocks_per_lane=bpl, tile_blocks=tile)
    try:
        A.aesgpu_batch_run(plan, d_keys, m, d_in, d_out)
        torch.cuda.synchronize()
    finally:
        A.aesgpu_batch_free(plan)
    return from_dev(d_out)


@pytest.mark.parametrize("bpl,tile", [(4, 8192), (2, 256), (1, 64)])
def test_noalloc_equals_planned_run_twice(A, ctx, bpl, tile):
    import torch
    rng = np.random.default_rng(700 + bpl)
    for call, (m, max_blocks) in enumerate([(400, 4096), (37, 300)]):
        msgs, keys, data, total = _batch(A, rng, m, max_blocks)
        log(f"case: noalloc call {call + 1}, {m} messages, {total} bytes, bpl={bpl} tile={tile}")
        d_keys = to_dev(keys.reshape(-1))
        d_in = to_dev(data)
        want = _planned(A, ctx, msgs, d_keys, m, d_in, total, bpl, tile)
        d_out = torch.full((total,), 0x5A, dtype=torch.uint8, device="cuda")
        A.aesgpu_batch_run_noalloc(ctx, msgs, d_keys, m, d_in, d_out, blocks_per_lane=bpl,
                                   tile_blocks=tile)
        torch.cuda.synchronize()
        got = from_dev(d_out)
        assert np.array_equal(got, want), f"call {call + 1}: noalloc output != planned run"


def test_noalloc_refuses_batch_larger_than_scratch(A, ctx):
    import torch
    m = A.AESGPU_NOALLOC_SCRATCH_BYTES // 64 + 1      # 64 descriptor bytes per message alone
    zeros = np.zeros(m, dtype=np.int64)
    msgs = A.make_msgs(16 * np.arange(m), 16 * np.arange(m), zeros + 16, zeros, zeros + 128,
                       zeros, zeros)
    d = torch.zeros(16 * m, dtype=torch.uint8, device="cuda")
    k = torch.zeros(32, dtype=torch.uint8, device="cuda")
    st = A.aesgpu_batch_run_noalloc(ctx, msgs, k, 1, d, d, check=False)
    assert st == A.AESGPU_ESCRATCH
    # A bad message is still reported as such, before the size check.
    bad = A.make_msgs([8], [0], [32], [0], [128], [0], [0])
    assert A.aesgpu_batch_run_noalloc(ctx, bad, k, 1, d, d, check=False) == A.AESGPU_EALIGN
    # An empty batch is a no-op.
    empty = A.make_msgs([0], [0], [0], [0], [128], [0], [0])
    assert A.aesgpu_batch_run_noalloc(ctx, empty, None, 0, None, None, 0, 0) == A.AESGPU_OK
