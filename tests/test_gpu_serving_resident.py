"""GPU tests of the server's resident mode (one kernel stays on the GPU and
takes tiles from rings in pinned host memory): every request's output equals
the oracle's, a request alone gives the same bytes as in the mix, a tiny
arena and a large request spread over many tiles keep outputs exact, the
kernel ends by itself when idle and is launched again for new requests, a
one-direction backlog moves the split of workgroups between the table sets,
destroying the server with work in flight returns promptly, and the trace
replay reports consistent timestamps."""
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
    return workloads.serving(rate_per_s=1000.0, n_requests=1200, seed=14, n_keys=64, lo=64,
                             hi=1 << 16, source_bytes=1 << 22)


def _expected(tr, j):
    k = int(tr.key_ids[j])
    key = tr.pool_keys[k, : tr.pool_bits[k] // 8]
    src = tr.source[tr.src_offsets[j]: tr.src_offsets[j] + tr.sizes[j]]
    return oracle.ecb(key, src, decrypt=bool(tr.dirs[j]))


def _drain(A, server, want, copies, timeout=60):
    """Polls until `want` requests finished; copies and releases outputs."""
    import torch
    got = 0
    deadline = time.time() + timeout
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
        time.sleep(0.0002)


def _server(A, ctx, tr, **kw):
    return A.aesgpu_server_create(ctx, tr.pool_keys, tr.pool_bits,
                                  flags=A.AESGPU_SERVER_RESIDENT, **kw)


def test_resident_mix_and_alone_match_oracle(A, ctx, pool):
    import torch
    tr = pool
    n = tr.sizes.size
    src = torch.from_numpy(tr.source.copy()).to("cuda")
    base = src.data_ptr()
    server = _server(A, ctx, tr, arena_bytes=64 << 20)
    try:
        log(f"case: resident, {n} requests submitted at once")
        mix = {}
        for j in range(n):
            A.aesgpu_server_submit(server, j, int(tr.dirs[j]), int(tr.key_ids[j]),
                                   base + int(tr.src_offsets[j]), int(tr.sizes[j]))
        _drain(A, server, n, mix)
        st = A.aesgpu_server_get_stats(server)
        log(f"kernel launches {st.batches}, most admitted at once {st.max_batch_requests}")
        assert st.requests_done == n and st.arena_used == 0 and st.batches >= 1
        for j in range(n):
            assert np.array_equal(mix[j], _expected(tr, j)), f"request {j} in the mix"
        log("case: resident, the same requests one at a time")
        alone = {}
        for j in range(300):
            A.aesgpu_server_submit(server, j, int(tr.dirs[j]), int(tr.key_ids[j]),
                                   base + int(tr.src_offsets[j]), int(tr.sizes[j]))
            _drain(A, server, 1, alone)
            assert np.array_equal(alone[j], mix[j]), f"request {j}: alone != in the mix"
    finally:
        A.aesgpu_server_destroy(server)


@pytest.mark.parametrize("bpl", [1, 2, 4])
def test_resident_tiny_arena(A, ctx, pool, bpl):
    """A 128 KiB arena forces slot and memory reuse; every blocks-per-lane
    variant of the kernel."""
    import torch
    tr = pool
    src = torch.from_numpy(tr.source.copy()).to("cuda")
    base = src.data_ptr()
    log(f"case: resident, 128 KiB arena, {bpl} blocks per lane")
    server = _server(A, ctx, tr, arena_bytes=1 << 17, blocks_per_lane=bpl)
    try:
        outs = {}
        n = 300
        for j in range(n):
            A.aesgpu_server_submit(server, j, int(tr.dirs[j]), int(tr.key_ids[j]),
                                   base + int(tr.src_offsets[j]), int(tr.sizes[j]))
        _drain(A, server, n, outs)
        assert A.aesgpu_server_get_stats(server).arena_high_water <= 1 << 17
        for j in range(n):
            assert np.array_equal(outs[j], _expected(tr, j)), f"request {j}"
    finally:
        A.aesgpu_server_destroy(server)


@pytest.mark.parametrize("tile_blocks", [0, 256])
def test_resident_large_requests(A, ctx, pool, tile_blocks):
    """16 MiB requests, alone (spread over every wave of their set) and four at
    once in both directions; sampled blocks against the oracle, and
    decrypt(encrypt(x)) = x on the whole buffer."""
    import torch
    tr = pool
    n = 16 << 20
    rng = np.random.default_rng(77 + tile_blocks)
    data = rng.integers(0, 256, n, dtype=np.uint8)
    src = torch.from_numpy(data).to("cuda")
    server = _server(A, ctx, tr, arena_bytes=256 << 20, tile_blocks=tile_blocks)
    try:
        log(f"case: resident, 16 MiB alone, tile_blocks={tile_blocks}")
        outs = {}
        A.aesgpu_server_submit(server, 0, 0, 5, src.data_ptr(), n)
        _drain(A, server, 1, outs)
        k = int(5)
        key = tr.pool_keys[k, : tr.pool_bits[k] // 8]
        idx = np.unique(np.concatenate([np.arange(4096), np.arange(n // 16 - 4096, n // 16),
                                        rng.integers(0, n // 16, 8192)]))
        got = outs[0].reshape(-1, 16)[idx]
        assert np.array_equal(got, oracle.ecb_sampled(key, data, idx))
        ct = torch.from_numpy(outs[0]).to("cuda")
        log("case: resident, four 16 MiB requests at once, both directions")
        A.aesgpu_server_submit(server, 1, 1, 5, ct.data_ptr(), n)      # decrypt the ciphertext
        A.aesgpu_server_submit(server, 2, 0, 9, src.data_ptr(), n)
        A.aesgpu_server_submit(server, 3, 1, 9, src.data_ptr(), n)
        A.aesgpu_server_submit(server, 4, 0, 5, src.data_ptr() + 16, n - 32)
        _drain(A, server, 4, outs)
        assert np.array_equal(outs[1], data), "decrypt(encrypt(x)) != x"
        key9 = tr.pool_keys[9, : tr.pool_bits[9] // 8]
        assert np.array_equal(outs[2].reshape(-1, 16)[idx], oracle.ecb_sampled(key9, data, idx))
        assert np.array_equal(outs[3].reshape(-1, 16)[idx],
                              oracle.ecb_sampled(key9, data, idx, decrypt=True))
        assert np.array_equal(outs[4], outs[0][16:n - 16])
    finally:
        A.aesgpu_server_destroy(server)


def test_resident_kernel_ends_when_idle_and_restarts(A, ctx, pool):
    import torch
    tr = pool
    src = torch.from_numpy(tr.source.copy()).to("cuda")
    base = src.data_ptr()
    server = _server(A, ctx, tr, arena_bytes=16 << 20)
    try:
        outs = {}
        for round_ in range(3):
            log(f"case: resident, idle gap {round_}")
            for j in range(20 * round_, 20 * round_ + 20):
                A.aesgpu_server_submit(server, j, int(tr.dirs[j]), int(tr.key_ids[j]),
                                       base + int(tr.src_offsets[j]), int(tr.sizes[j]))
            _drain(A, server, 20, outs)
            launches = A.aesgpu_server_get_stats(server).batches
            assert launches == round_ + 1, f"{launches} launches after {round_ + 1} bursts"
            time.sleep(1.0)   # well past the kernel's idle limit
        for j in range(60):
            assert np.array_equal(outs[j], _expected(tr, j)), f"request {j}"
    finally:
        A.aesgpu_server_destroy(server)


def test_resident_rebalances_one_direction_backlog(A, ctx, pool):
    """A large one-direction backlog makes the server stop the kernel and
    launch it with more workgroups on that direction's tables; every output
    is still exact (sampled against the oracle, then round-tripped through a
    decryption backlog, which moves the split back)."""
    import torch
    tr = pool
    n = 16 << 20
    m = 48                      # 48 x 16 MiB = 48 M blocks of one direction
    rng = np.random.default_rng(91)
    data = rng.integers(0, 256, n, dtype=np.uint8)
    src = torch.from_numpy(data).to("cuda")
    server = _server(A, ctx, tr, arena_bytes=2 << 30)
    try:
        log("case: resident, encryption-only backlog behind a kernel split half and half")
        outs = {}
        # A small request starts the kernel at the even split; the backlog
        # comes while it runs (it stays up for tens of milliseconds idle).
        A.aesgpu_server_submit(server, 10_000, 1, 3, src.data_ptr(), 1 << 16)
        _drain(A, server, 1, {})
        time.sleep(0.005)
        for j in range(m):
            A.aesgpu_server_submit(server, j, 0, j % 64, src.data_ptr(), n)
        _drain(A, server, m, outs)
        st = A.aesgpu_server_get_stats(server)
        log(f"launches {st.batches}, rebalances {st.rebalances}")
        assert st.rebalances >= 1 and st.batches >= 2, "the split did not change"
        idx = np.unique(np.concatenate([np.arange(1024), rng.integers(0, n // 16, 2048)]))
        for j in (0, 1, m - 1):
            key = tr.pool_keys[j % 64, : tr.pool_bits[j % 64] // 8]
            assert np.array_equal(outs[j].reshape(-1, 16)[idx], oracle.ecb_sampled(key, data, idx))
        log("case: resident, decryption-only backlog of the ciphertexts")
        cts = [torch.from_numpy(outs[j]).to("cuda") for j in range(m)]
        back = {}
        for j in range(m):
            A.aesgpu_server_submit(server, m + j, 1, j % 64, cts[j].data_ptr(), n)
        _drain(A, server, m, back)
        for j in range(m):
            assert np.array_equal(back[m + j], data), f"request {j}: decrypt(encrypt(x)) != x"
    finally:
        A.aesgpu_server_destroy(server)


def test_resident_destroy_with_work_in_flight(A, ctx, pool):
    """Destroying the server while requests are queued and running stops the
    kernel (queued tiles are dropped) and returns promptly; a new server on
    the same context then works."""
    import torch
    tr = pool
    n = 16 << 20
    src = torch.zeros(n, dtype=torch.uint8, device="cuda")
    server = _server(A, ctx, tr, arena_bytes=2 << 30)
    for j in range(100):
        A.aesgpu_server_submit(server, j, j % 2, j % 64, src.data_ptr(), n)
    time.sleep(0.002)
    t0 = time.time()
    A.aesgpu_server_destroy(server)
    log(f"destroy with work in flight took {(time.time() - t0) * 1e3:.1f} ms")
    assert time.time() - t0 < 5.0
    torch.cuda.synchronize()
    server = _server(A, ctx, tr, arena_bytes=16 << 20)
    try:
        outs = {}
        base = torch.from_numpy(tr.source.copy()).to("cuda")
        for j in range(10):
            A.aesgpu_server_submit(server, j, int(tr.dirs[j]), int(tr.key_ids[j]),
                                   base.data_ptr() + int(tr.src_offsets[j]), int(tr.sizes[j]))
        _drain(A, server, 10, outs)
        for j in range(10):
            assert np.array_equal(outs[j], _expected(tr, j)), f"request {j}"
    finally:
        A.aesgpu_server_destroy(server)


def test_resident_replay_poisson_trace(A, ctx):
    import torch
    from paper_1201_0398_amd import workloads
    tr = workloads.serving(rate_per_s=20000.0, n_requests=4000, seed=15, n_keys=64, lo=64,
                           hi=1 << 20, source_bytes=1 << 24)
    src = torch.from_numpy(tr.source.copy()).to("cuda")
    server = _server(A, ctx, tr, arena_bytes=1 << 28)
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
        log(f"resident replay: p50 {np.median(lat) * 1e6:.0f} us, "
            f"p99 {np.quantile(lat, 0.99) * 1e6:.0f} us")
        assert A.aesgpu_server_get_stats(server).arena_used == 0
    finally:
        A.aesgpu_server_destroy(server)


def test_resident_steady_trickle_every_request_completes(A, ctx, pool):
    """Light steady traffic: one 4 KiB request every 2..5 ms for about three
    seconds, so the kernel stays up (each new tail restarts its idle count)
    while most of its waves have nothing to do for seconds.  Every request
    must finish within a deadline and equal the oracle's output (a wave that
    left on a timer of its own while holding a ticket, or every worker of a
    set leaving while the set's poller still ran, would strand a request)."""
    import torch
    tr = pool
    src = torch.from_numpy(tr.source.copy()).to("cuda")
    base = src.data_ptr()
    rng = np.random.default_rng(123)
    n = 800
    dirs = rng.integers(0, 2, n)
    keys = rng.integers(0, 64, n)
    offs = 16 * rng.integers(0, (tr.source.size - 4096) // 16, n)
    gaps = rng.uniform(0.002, 0.005, n)
    server = _server(A, ctx, tr, arena_bytes=16 << 20)
    log(f"case: resident, trickle of {n} 4 KiB requests, 2..5 ms apart")
    try:
        outs, t_sub, t_got = {}, {}, {}
        j = 0
        next_t = time.time()
        deadline = time.time() + gaps.sum() + 30.0
        while len(outs) < n:
            now = time.time()
            assert now < deadline, f"{n - len(outs)} requests never finished"
            if j < n and now >= next_t:
                A.aesgpu_server_submit(server, j, int(dirs[j]), int(keys[j]), base + int(offs[j]),
                                       4096)
                t_sub[j] = time.time()
                next_t = t_sub[j] + gaps[j]
                j += 1
            for d in A.aesgpu_server_poll(server):
                assert d.status == 0, f"request {d.req_id} failed: {d.status}"
                out = torch.empty(d.n_bytes, dtype=torch.uint8, device="cuda")
                copy_device(out.data_ptr(), d.d_out, d.n_bytes)
                outs[d.req_id] = from_dev(out)
                t_got[d.req_id] = time.time()
                A.aesgpu_server_release(server, d.d_out, d.n_bytes)
            pending = [q for q in range(max(0, j - 64), j) if q not in t_got]
            if pending:
                q = pending[0]
                assert time.time() - t_sub[q] < 2.0, f"request {q} stranded"
            time.sleep(0.0002)
        lat = np.array([t_got[q] - t_sub[q] for q in range(n)])
        st = A.aesgpu_server_get_stats(server)
        log(f"trickle: kernel launches {st.batches}, latency p50 {np.median(lat) * 1e3:.2f} ms, "
            f"max {lat.max() * 1e3:.2f} ms")
        for q in range(n):
            k = int(keys[q])
            key = tr.pool_keys[k, : tr.pool_bits[k] // 8]
            want = oracle.ecb(key, tr.source[offs[q]: offs[q] + 4096], decrypt=bool(dirs[q]))
            assert np.array_equal(outs[q], want), f"request {q}"
    finally:
        A.aesgpu_server_destroy(server)
