"""The launch-shape autotuner: cache keys and persistence on the CPU, and on
the GPU a tuned plan that still matches the oracle and a second call that is
served from the cache."""
import numpy as np
import pytest

import oracle
from gpu_common import from_dev, requires_gpu, to_dev
from paper_1201_0398_amd import autotune


def test_workload_key_buckets():
    k1 = autotune.workload_key("gfx950", [1024, 2048], [0, 0], [0, 1])
    k2 = autotune.workload_key("gfx950", [1100, 2100], [0, 0], [0, 1])
    k3 = autotune.workload_key("gfx950", [1024, 2048], [0, 1], [0, 1])
    assert k1 == k2                      # same buckets
    assert k1 != k3                      # CTR messages never need the inverse tables
    assert k1.startswith("gfx950|") and "inv7" in k1
    assert autotune.workload_key("gfx950", [0], [0], [0]).endswith("empty")


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(p) == {}
    autotune.store_cache({"k": {"blocks_per_lane": 2, "tile_blocks": 4096}}, p)
    assert autotune.load_cache(p)["k"]["tile_blocks"] == 4096
    (tmp_path / "bad.json").write_text("not json")
    assert autotune.load_cache(str(tmp_path / "bad.json")) == {}


@pytest.mark.gpu
@requires_gpu
def test_tuned_plan_is_correct_and_cached(tmp_path):
    import torch
    from paper_1201_0398_amd import aesgpu as A
    ctx = A.aesgpu_create()
    try:
        rng = np.random.default_rng(77)
        m = 64
        lengths = 16 * rng.integers(1, 4096, size=m)
        modes = rng.integers(0, 2, size=m)
        dirs = rng.integers(0, 2, size=m)
        bits = np.array([128, 192, 256])[rng.integers(0, 3, size=m)]
        offs = np.concatenate([[0], np.cumsum(lengths)[:-1]])
        keys = rng.integers(0, 256, (m, 32), dtype=np.uint8)
        nonces = rng.integers(0, 256, (m, 12), dtype=np.uint8)
        data = rng.integers(0, 256, int(lengths.sum()), dtype=np.uint8)
        msgs = A.make_msgs(offs, offs, lengths, np.arange(m), bits, modes, dirs, nonces)
        d_keys, d_in = to_dev(keys.reshape(-1)), to_dev(data)
        d_out = torch.empty_like(d_in)
        path = str(tmp_path / "tune.json")
        cands = [(1, 1024), (2, 2048), (2, 8192)]
        c1 = autotune.tune_batch(ctx, msgs, lengths, modes, dirs, d_keys, m, d_in, d_out,
                                 candidates=cands, reps=2, path=path)
        assert (c1.blocks_per_lane, c1.tile_blocks) in cands and not c1.from_cache
        assert len(c1.timings) == 3
        c2 = autotune.tune_batch(ctx, msgs, lengths, modes, dirs, d_keys, m, d_in, d_out,
                                 candidates=cands, path=path)
        assert c2.from_cache and (c2.blocks_per_lane, c2.tile_blocks) == \
            (c1.blocks_per_lane, c1.tile_blocks)
        plan = A.aesgpu_batch_plan(ctx, msgs, blocks_per_lane=c1.blocks_per_lane,
                                   tile_blocks=c1.tile_blocks)
        out = torch.zeros_like(d_in)
        A.aesgpu_batch_run(plan, d_keys, m, d_in, out)
        got = from_dev(out)
        A.aesgpu_batch_free(plan)
        for j in range(m):
            o, L = int(offs[j]), int(lengths[j])
            key = keys[j, : bits[j] // 8]
            want = (oracle.ctr(key, nonces[j], 1, data[o:o + L]) if modes[j]
                    else oracle.ecb(key, data[o:o + L], decrypt=bool(dirs[j])))
            assert np.array_equal(got[o:o + L], want), f"message {j}"
    finally:
        A.aesgpu_destroy(ctx)
