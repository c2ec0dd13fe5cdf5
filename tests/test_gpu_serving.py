"""GPU tests of the continuous-batching server: every request's output equals
the oracle's, the same request run alone gives the same bytes as in the mix
(zero tolerance), for small requests and over the served workload's whole
64 B .. 16 MiB size range, a tiny arena forces slot reuse without corrupting
outputs, and the trace replay reports consistent timestamps."""
import time

import numpy as np
import pytest

import oracle
from gpu_common import copy_device, from_dev, log, requires_gpu

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


@pytest.fixture(scope="module")
def pool():
    from paper_1201_0398_amd import workloads
    tr = workloads.serving(rate_per_s=1000.0, n_requests=1200, seed=4, n_keys=64, lo=64,
                           hi=1 << 16, source_bytes=1 << 22)
    return tr


def _expected(tr, j):
    k = int(tr.key_ids[j])
    key = tr.pool_keys[k, : tr.pool_bits[k] // 8]
    src = tr.source[tr.src_offsets[j]: tr.src_offsets[j] + tr.sizes[j]]
    return oracle.ecb(key, src, decrypt=bool(tr.dirs[j]))


def _drain(A, server, want, copies):
    """Polls until `want` requests finished; copies and releases outputs."""
    import torch
    got = 0
    deadline = time.time() + 60
    while got < want:
        assert time.time() < deadline, "server did not finish in time"
        for d in A.aesgpu_server_poll(server):
            assert d.status == 0, f"request {d.req_id} failed: {d.status}"
            assert d.t_arrival <= d.t_launch + 1e-9 and d.t_launch <= d.t_done
            out = torch.empty(d.n_bytes, dtype=torch.uint8, device="cuda")
            copy_device(out.data_ptr(), d.d_out, d.n_bytes)   # out of the arena first
            copies[d.req_id] = from_dev(out)
            A.aesgpu_server_release(server, d.d_out, d.n_bytes)
            got += 1
        time.sleep(0.0005)


@pytest.mark.parametrize("direct", ["default", "never"])
def test_in_mix_and_alone_match_oracle(A, ctx, pool, direct):
    """Alone, a request is a batch of one: a single-buffer launch by default,
    the batched kernel when direct launches are off."""
    import torch
    tr = pool
    n = tr.sizes.size
    src = torch.from_numpy(tr.source.copy()).to("cuda")
    base = src.data_ptr()
    server = A.aesgpu_server_create(
        ctx, tr.pool_keys, tr.pool_bits, arena_bytes=64 << 20,
        direct_requests=A.AESGPU_SERVER_NO_DIRECT if direct == "never" else 0)
    try:
        log(f"case: {n} requests submitted at once (in the mix), direct={direct}")
        mix = {}
        for j in range(n):
            A.aesgpu_server_submit(server, j, int(tr.dirs[j]), int(tr.key_ids[j]),
                                   base + int(tr.src_offsets[j]), int(tr.sizes[j]))
        _drain(A, server, n, mix)
        st = A.aesgpu_server_get_stats(server)
        log(f"batches {st.batches}, max batch {st.max_batch_requests}")
        assert st.requests_done == n and st.arena_used == 0
        for j in range(n):
            assert np.array_equal(mix[j], _expected(tr, j)), f"request {j} in the mix"
        log("case: the same requests one at a time (alone)")
        alone = {}
        for j in range(1000):
            A.aesgpu_server_submit(server, j, int(tr.dirs[j]), int(tr.key_ids[j]),
                                   base + int(tr.src_offsets[j]), int(tr.sizes[j]))
            _drain(A, server, 1, alone)
            assert np.array_equal(alone[j], mix[j]), f"request {j}: alone != in the mix"
    finally:
        A.aesgpu_server_destroy(server)


@pytest.mark.parametrize("direct", [0, 16])
def test_tiny_arena_forces_reuse(A, ctx, pool, direct):
    """Batches of up to 7 requests in a 128 KiB arena; with direct=16 every
    batch runs as single-buffer launches, one per request."""
    import torch
    tr = pool
    src = torch.from_numpy(tr.source.copy()).to("cuda")
    base = src.data_ptr()
    log(f"case: tiny arena, direct={direct}")
    server = A.aesgpu_server_create(ctx, tr.pool_keys, tr.pool_bits, arena_bytes=1 << 17,
                                    max_batch_requests=7, direct_requests=direct)
    try:
        outs = {}
        n = 300
        for j in range(n):
            A.aesgpu_server_submit(server, j, int(tr.dirs[j]), int(tr.key_ids[j]),
                                   base + int(tr.src_offsets[j]), int(tr.sizes[j]))
        _drain(A, server, n, outs)
        st = A.aesgpu_server_get_stats(server)
        assert st.arena_high_water <= 1 << 17 and st.batches >= n // 7
        for j in range(n):
            assert np.array_equal(outs[j], _expected(tr, j)), f"request {j}"
        # Argument errors.
        assert A.aesgpu_server_submit(server, 0, 0, 0, base, 1 << 18, check=False) == \
            A.AESGPU_EINVAL                                   # larger than the arena
        assert A.aesgpu_server_submit(server, 0, 0, 0, base + 8, 64, check=False) == \
            A.AESGPU_EALIGN
        assert A.aesgpu_server_submit(server, 0, 0, 64, base, 64, check=False) == A.AESGPU_EINVAL
        assert A.aesgpu_server_submit(server, 0, 2, 0, base, 64, check=False) == A.AESGPU_EINVAL
        assert A.aesgpu_server_submit(server, 0, 0, 0, base, 24, check=False) == A.AESGPU_EINVAL
    finally:
        A.aesgpu_server_destroy(server)


def test_server_config_errors(A, ctx, pool):
    import ctypes
    tr = pool
    L = A.lib()
    out = ctypes.c_void_p()
    keys = np.ascontiguousarray(tr.pool_keys)
    bits = np.ascontiguousarray(tr.pool_bits, dtype=np.uint16)
    for bad in [dict(direct_requests=17), dict(n_streams=9), dict(blocks_per_lane=3),
                dict(arena_bytes=100), dict(tile_blocks=100)]:
        kw = dict(arena_bytes=1 << 20)
        kw.update(bad)
        cfg = A.aesgpu_server_config(kw.pop("arena_bytes"), kw.get("n_streams", 0),
                                     kw.get("blocks_per_lane", 0), kw.get("tile_blocks", 0),
                                     0, 0, 0, kw.get("direct_requests", 0))
        st = L.aesgpu_server_create(ctx, keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                    bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                    bits.size, ctypes.byref(cfg), ctypes.byref(out))
        assert st == A.AESGPU_EINVAL, bad
        assert not out.value


def test_replay_poisson_trace(A, ctx, pool):
    import torch
    from paper_1201_0398_amd import workloads
    tr = workloads.serving(rate_per_s=20000.0, n_requests=4000, seed=5, n_keys=64, lo=64,
                           hi=1 << 20, source_bytes=1 << 24)
    src = torch.from_numpy(tr.source.copy()).to("cuda")
    server = A.aesgpu_server_create(ctx, tr.pool_keys, tr.pool_bits, arena_bytes=1 << 28)
    try:
        reqs = A.make_requests(tr.arrivals, src.data_ptr() + tr.src_offsets, tr.sizes,
                               tr.key_ids, tr.dirs)
        t0 = A.aesgpu_server_now(server) + 0.01
        done = A.aesgpu_server_replay(server, reqs, t0)
        arr = np.array([(d.req_id, d.t_arrival, d.t_launch, d.t_done) for d in done])
        assert (arr[:, 0] == np.arange(4000)).all()
        assert np.allclose(arr[:, 1], t0 + tr.arrivals)
        assert (arr[:, 2] >= arr[:, 1] - 1e-9).all() and (arr[:, 3] >= arr[:, 2]).all()
        lat = arr[:, 3] - arr[:, 1]
        log(f"replay: p50 {np.median(lat) * 1e6:.0f} us, p99 {np.quantile(lat, 0.99) * 1e6:.0f} us")
        assert A.aesgpu_server_get_stats(server).arena_used == 0
    finally:
        A.aesgpu_server_destroy(server)


@pytest.fixture(scope="module")
def full_range():
    """Requests over the served workload's whole size range, 64 B .. 16 MiB
    log-uniform, half encrypt and half decrypt, and the oracle's output for
    every one of them."""
    from paper_1201_0398_amd import workloads
    tr = workloads.serving(rate_per_s=1000.0, n_requests=160, seed=24, n_keys=64, lo=64,
                           hi=1 << 24, source_bytes=1 << 26)
    log(f"oracle over {int(tr.sizes.sum())} bytes of requests up to {int(tr.sizes.max())} B")
    return tr, [_expected(tr, j) for j in range(tr.sizes.size)]


@pytest.mark.parametrize("direct", ["default", "never"])
def test_full_size_range_in_mix_and_alone(A, ctx, full_range, direct):
    """The batched server over 64 B .. 16 MiB requests: every output in the
    mix equals the oracle's, and requests run alone (the 12 largest and 28
    others) give the same bytes as in the mix."""
    import torch
    tr, want = full_range
    n = tr.sizes.size
    src = torch.from_numpy(tr.source.copy()).to("cuda")
    base = src.data_ptr()
    server = A.aesgpu_server_create(
        ctx, tr.pool_keys, tr.pool_bits, arena_bytes=1 << 30,
        direct_requests=A.AESGPU_SERVER_NO_DIRECT if direct == "never" else 0)
    try:
        log(f"case: {n} requests of 64 B..16 MiB at once, direct={direct}")
        mix = {}
        for j in range(n):
            A.aesgpu_server_submit(server, j, int(tr.dirs[j]), int(tr.key_ids[j]),
                                   base + int(tr.src_offsets[j]), int(tr.sizes[j]))
        _drain(A, server, n, mix)
        assert A.aesgpu_server_get_stats(server).arena_used == 0
        for j in range(n):
            assert np.array_equal(mix[j], want[j]), f"request {j} ({tr.sizes[j]} B) in the mix"
        order = np.argsort(tr.sizes)
        alone_ids = np.unique(np.concatenate([order[-12:], np.arange(28)]))
        log(f"case: {alone_ids.size} of them alone, direct={direct}")
        for j in alone_ids:
            alone = {}
            A.aesgpu_server_submit(server, int(j), int(tr.dirs[j]), int(tr.key_ids[j]),
                                   base + int(tr.src_offsets[j]), int(tr.sizes[j]))
            _drain(A, server, 1, alone)
            assert np.array_equal(alone[int(j)], mix[int(j)]), f"request {j}: alone != in the mix"
    finally:
        A.aesgpu_server_destroy(server)
