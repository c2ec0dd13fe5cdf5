"""GPU parity of the batched persistent launch: every message of a mixed batch
(own key, key size, mode, direction, uneven length) against the CPU oracle run
on that message alone; graph replays against direct launches; the full
65,536-message workload compared in full with the oracle in both directions
(digests of the whole outputs) plus the whole-batch round trip."""
import numpy as np
import pytest

import oracle
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


def _random_batch(rng, m, max_len=1 << 16, gap=True):
    lengths = 16 * rng.integers(1, max_len // 16 + 1, size=m)
    modes = rng.integers(0, 2, size=m)
    ctr_tail = rng.integers(0, 16, size=m)
    lengths = np.where(modes == 1, np.maximum(lengths - ctr_tail, 1), lengths)
    bits = np.array([128, 192, 256])[rng.integers(0, 3, size=m)]
    dirs = rng.integers(0, 2, size=m)
    # Pack with optional gaps, 16-byte aligned; outputs at different offsets.
    pad = 16 * rng.integers(0, 3, size=m) if gap else np.zeros(m, dtype=np.int64)
    span = 16 * ((lengths + 15) // 16) + pad
    in_off = np.concatenate([[0], np.cumsum(span)[:-1]])
    out_off = np.concatenate([[0], np.cumsum(span[::-1])[:-1]])[::-1].copy()
    keys = np.zeros((m, 32), dtype=np.uint8)
    for j in range(m):
        keys[j, : bits[j] // 8] = rng.integers(0, 256, bits[j] // 8, dtype=np.uint8)
    nonces = rng.integers(0, 256, (m, 12), dtype=np.uint8)
    ctr0 = rng.integers(0, 1 << 31, size=m).astype(np.uint32)
    total = int(span.sum())
    data = rng.integers(0, 256, total, dtype=np.uint8)
    return dict(lengths=lengths, modes=modes, bits=bits, dirs=dirs, in_off=in_off,
                out_off=out_off, keys=keys, nonces=nonces, ctr0=ctr0, data=data, total=total)


def _expected(b, j):
    L = int(b["lengths"][j])
    key = b["keys"][j, : b["bits"][j] // 8]
    src = b["data"][b["in_off"][j]: b["in_off"][j] + L]
    if b["modes"][j] == 1:
        return oracle.ctr(key, b["nonces"][j], int(b["ctr0"][j]), src)
    return oracle.ecb(key, src, decrypt=bool(b["dirs"][j]))


def _plan(A, ctx, b, **kw):
    msgs = A.make_msgs(b["in_off"], b["out_off"], b["lengths"], np.arange(len(b["lengths"])),
                       b["bits"], b["modes"], b["dirs"], b["nonces"], b["ctr0"])
    return A.aesgpu_batch_plan(ctx, msgs, **kw)


@pytest.mark.parametrize("bpl,tile", [(1, 2048), (2, 128), (2, 8192), (1, 64), (4, 256), (4, 8192)])
def test_mixed_batch_matches_oracle(A, ctx, bpl, tile):
    import torch
    rng = np.random.default_rng(30 + bpl + tile)
    b = _random_batch(rng, 300)
    log(f"case: mixed batch of 300, bpl={bpl} tile={tile}, {b['total']} bytes")
    plan = _plan(A, ctx, b, blocks_per_lane=bpl, tile_blocks=tile)
    try:
        st = A.aesgpu_batch_info(plan)
        assert st.n_msgs == 300 and st.launches == 1
        assert st.n_tiles_forward > 0 and st.n_tiles_inverse > 0
        d_keys = to_dev(b["keys"].reshape(-1))
        d_in = to_dev(b["data"])
        d_out = torch.full((b["total"],), 0x5A, dtype=torch.uint8, device="cuda")
        A.aesgpu_batch_run(plan, d_keys, 300, d_in, d_out)
        out = from_dev(d_out)
        covered = np.zeros(b["total"], dtype=bool)
        for j in range(300):
            o, L = int(b["out_off"][j]), int(b["lengths"][j])
            assert np.array_equal(out[o:o + L], _expected(b, j)), f"message {j}"
            covered[o:o + L] = True
        assert (out[~covered] == 0x5A).all(), "wrote outside the messages"
    finally:
        A.aesgpu_batch_free(plan)


@pytest.mark.parametrize("bpl,tile", [(1, 64), (2, 128), (4, 256), (4, 512), (2, 8192)])
def test_ctr_counter_alignment_in_batches(A, ctx, bpl, tile):
    """CTR messages whose first counter sits at every kind of offset from the
    kernel's step (64 * blocks per lane): 0, 1, one short of a step, a step,
    255, 256, random, and the largest counter that still fits 32 bits; lengths
    from one partial block to several tiles, with and without a partial last
    block.  Every byte must match the oracle and nothing outside the
    messages may change."""
    import torch
    rng = np.random.default_rng(77 + bpl + tile)
    step = 64 * bpl
    starts = [0, 1, step - 1, step, step + 1, 255, 256, 257, 3 * step - 5]
    lens = [5, 16, 16 * step - 16, 16 * step, 16 * step + 9, 16 * (tile + step) + 3,
            16 * 3 * tile + 7, 16 * 2 * tile]
    ctr0s, lengths = [], []
    for c in starts:
        for L in lens:
            ctr0s.append(c + int(rng.integers(0, 1 << 20)) * 256)
            lengths.append(L)
    # Largest first counters: the message's last block uses counter 2^32 - 1.
    for L in (16 * step + 9, 16 * (tile + 1), 16):
        lengths.append(L)
        ctr0s.append((1 << 32) - (L + 15) // 16)
    m = len(lengths)
    lengths = np.array(lengths)
    span = 16 * ((lengths + 15) // 16) + 16
    in_off = np.concatenate([[0], np.cumsum(span)[:-1]])
    out_off = in_off.copy()
    bits = np.array([128, 192, 256])[rng.integers(0, 3, size=m)]
    keys = np.zeros((m, 32), dtype=np.uint8)
    for j in range(m):
        keys[j, : bits[j] // 8] = rng.integers(0, 256, bits[j] // 8, dtype=np.uint8)
    nonces = rng.integers(0, 256, (m, 12), dtype=np.uint8)
    ctr0 = np.array(ctr0s, dtype=np.uint64)
    total = int(span.sum())
    data = rng.integers(0, 256, total, dtype=np.uint8)
    log(f"case: {m} CTR messages, bpl={bpl} tile={tile}, {total} bytes")
    msgs = A.make_msgs(in_off, out_off, lengths, np.arange(m), bits, np.ones(m, dtype=np.int64),
                       np.zeros(m, dtype=np.int64), nonces, ctr0)
    plan = A.aesgpu_batch_plan(ctx, msgs, blocks_per_lane=bpl, tile_blocks=tile)
    try:
        d_out = torch.full((total,), 0x5A, dtype=torch.uint8, device="cuda")
        A.aesgpu_batch_run(plan, to_dev(keys.reshape(-1)), m, to_dev(data), d_out)
        out = from_dev(d_out)
        covered = np.zeros(total, dtype=bool)
        for j in range(m):
            o, L = int(out_off[j]), int(lengths[j])
            key = keys[j, : bits[j] // 8]
            want = oracle.ctr(key, nonces[j], int(ctr0[j]), data[o:o + L])
            assert np.array_equal(out[o:o + L], want), \
                f"message {j}: ctr0 {int(ctr0[j])} (mod step {int(ctr0[j]) % step}) len {L}"
            covered[o:o + L] = True
        assert (out[~covered] == 0x5A).all(), "wrote outside the messages"
    finally:
        A.aesgpu_batch_free(plan)


@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_many_short_messages_pull_runs(A, ctx, direction):
    """65,536 one-tile messages (1..4 blocks each, own key each): far more
    tiles than waves, so waves pull runs of several tiles per atomic (the run
    length is computed below as the launch computes it).  Forward: ECB
    encryption and CTR (with partial last blocks); inverse: ECB and CBC
    decryption.  Every message against the oracle."""
    import torch
    rng = np.random.default_rng(4242 + (direction == "inverse"))
    m = 65536
    n_cu = A.aesgpu_ctx_num_cus(ctx)
    grid = min((m + 15) // 16, n_cu, 1024)
    run = min(32, max(1, (m - 16 * grid) // (16 * grid * 4)))
    log(f"case: {m} short messages, {direction} queue, {run} tiles per pull")
    assert run > 1, "the case must exercise multi-tile pulls"
    blocks = rng.integers(1, 5, size=m)
    if direction == "forward":
        modes = rng.integers(0, 2, size=m)                   # ECB or CTR
        dirs = np.zeros(m, dtype=np.int64)
        lengths = np.where(modes == 1, 16 * blocks - rng.integers(0, 16, size=m), 16 * blocks)
    else:
        modes = np.where(rng.integers(0, 2, size=m) == 1, 2, 0)  # ECB or CBC
        dirs = np.ones(m, dtype=np.int64)
        lengths = 16 * blocks
    bits = np.array([128, 192, 256])[rng.integers(0, 3, size=m)]
    span = 16 * blocks
    offs = np.concatenate([[0], np.cumsum(span)[:-1]])
    keys = rng.integers(0, 256, (m, 32), dtype=np.uint8)
    nonces = rng.integers(0, 256, (m, 12), dtype=np.uint8)
    ctr0 = rng.integers(0, 1 << 31, size=m).astype(np.uint32)
    ivs = rng.integers(0, 256, (m, 16), dtype=np.uint8)
    total = int(span.sum())
    data = rng.integers(0, 256, total, dtype=np.uint8)
    msgs = A.make_msgs(offs, offs, lengths, np.arange(m), bits, modes, dirs, nonces, ctr0, iv=ivs)
    plan = A.aesgpu_batch_plan(ctx, msgs, blocks_per_lane=4, tile_blocks=8192)
    try:
        d_out = torch.zeros(total, dtype=torch.uint8, device="cuda")
        A.aesgpu_batch_run(plan, to_dev(keys.reshape(-1)), m, to_dev(data), d_out)
        out = from_dev(d_out)
    finally:
        A.aesgpu_batch_free(plan)
    for j in range(m):
        o, L = int(offs[j]), int(lengths[j])
        key = keys[j, : bits[j] // 8]
        src = data[o:o + L]
        if modes[j] == 1:
            want = oracle.ctr(key, nonces[j], int(ctr0[j]), src, threads=1)
        elif modes[j] == 2:
            want = oracle.cbc_decrypt(key, ivs[j], src, threads=1)
        else:
            want = oracle.ecb(key, src, decrypt=bool(dirs[j]), threads=1)
        assert np.array_equal(out[o:o + L], want), \
            f"message {j}: mode {modes[j]} bits {bits[j]} len {L}"


def test_graph_replays_match_direct_launch(A, ctx):
    import torch
    rng = np.random.default_rng(41)
    b = _random_batch(rng, 120, max_len=1 << 14)
    d_keys = to_dev(b["keys"].reshape(-1))
    d_in = to_dev(b["data"])
    direct = _plan(A, ctx, b, flags=A.AESGPU_BATCH_NO_GRAPH)
    graph = _plan(A, ctx, b)
    try:
        ref = torch.zeros(b["total"], dtype=torch.uint8, device="cuda")
        A.aesgpu_batch_run(direct, d_keys, 120, d_in, ref)
        torch.cuda.synchronize()
        for rep in range(4):
            out = torch.zeros_like(ref)
            A.aesgpu_batch_run(graph, d_keys, 120, d_in, out)
            junk = torch.randint(0, 256, (1 << 20,), device="cuda", dtype=torch.uint8)
            junk.sum()  # unrelated eager work between replays
            torch.cuda.synchronize()
            assert torch.equal(out, ref), f"graph replay {rep} differs"
        # New buffers force a re-capture.
        d_in2 = d_in.clone()
        out2 = torch.zeros_like(ref)
        A.aesgpu_batch_run(graph, d_keys, 120, d_in2, out2)
        assert torch.equal(out2, ref)
    finally:
        A.aesgpu_batch_free(direct)
        A.aesgpu_batch_free(graph)


def test_in_place_and_round_trip(A, ctx):
    import torch
    rng = np.random.default_rng(42)
    b = _random_batch(rng, 200, gap=False)
    b["out_off"] = b["in_off"]
    d_keys = to_dev(b["keys"].reshape(-1))
    d = to_dev(b["data"])
    enc = dict(b, dirs=np.zeros_like(b["dirs"]))
    dec = dict(b, dirs=np.ones_like(b["dirs"]))
    pe, pd = _plan(A, ctx, enc), _plan(A, ctx, dec)
    try:
        A.aesgpu_batch_run(pe, d_keys, 200, d, d)
        A.aesgpu_batch_run(pd, d_keys, 200, d, d)
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(d), b["data"]), "decrypt(encrypt(batch)) != batch"
    finally:
        A.aesgpu_batch_free(pe)
        A.aesgpu_batch_free(pd)


def _nb(t):
    return t.numel() * t.element_size()


def test_plan_and_run_errors(A, ctx):
    import torch
    rng = np.random.default_rng(43)
    b = _random_batch(rng, 8)
    msgs = A.make_msgs(b["in_off"], b["out_off"], b["lengths"], np.arange(8), b["bits"],
                       b["modes"], b["dirs"], b["nonces"], b["ctr0"])
    ok = A.aesgpu_batch_plan(ctx, msgs)
    try:
        d_keys = to_dev(b["keys"].reshape(-1))
        d_in = to_dev(b["data"])
        d_out = torch.empty_like(d_in)
        assert A.aesgpu_batch_run(ok, d_keys, 7, d_in, d_out, check=False) == A.AESGPU_EINVAL
        need = A.aesgpu_batch_info(ok)
        assert A.aesgpu_batch_run(ok, d_keys, 8, d_in, d_out, in_bytes=need.in_bytes_needed - 1,
                                  check=False) == A.AESGPU_EINVAL
        assert A.aesgpu_batch_run(ok, d_keys, 8, d_in, d_out, out_bytes=need.out_bytes_needed - 1,
                                  check=False) == A.AESGPU_EINVAL
        assert A.aesgpu_batch_run(ok, d_keys, 8, d_in.data_ptr() + 8, d_out,
                                  in_bytes=b["total"] - 8, check=False) == A.AESGPU_EALIGN
        # sizes beyond the tensors are refused by the binding
        with pytest.raises(ValueError):
            A.aesgpu_batch_run(ok, d_keys, 9, d_in, d_out)
        with pytest.raises(ValueError):
            A.aesgpu_batch_run(ok, d_keys, 8, d_in, d_out, in_bytes=_nb(d_in) + 16)
        with pytest.raises(ValueError):
            A.aesgpu_batch_run(ok, d_keys, 8, d_in, d_out, out_bytes=_nb(d_out) + 16)
    finally:
        A.aesgpu_batch_free(ok)
    bad = A.make_msgs([0], [0], [32], [0], [130], [0], [0])
    assert A.aesgpu_batch_plan(ctx, bad, check=False) == A.AESGPU_EKEYLEN
    bad = A.make_msgs([8], [0], [32], [0], [128], [0], [0])
    assert A.aesgpu_batch_plan(ctx, bad, check=False) == A.AESGPU_EALIGN
    bad = A.make_msgs([0], [0], [33], [0], [128], [0], [0])
    assert A.aesgpu_batch_plan(ctx, bad, check=False) == A.AESGPU_EINVAL
    bad = A.make_msgs([0], [0], [64], [0], [128], [1], [0], ctr0=[(1 << 32) - 2])
    assert A.aesgpu_batch_plan(ctx, bad, check=False) == A.AESGPU_ECTR_OVERFLOW
    assert A.aesgpu_batch_plan(ctx, bad, tile_blocks=100, check=False) == A.AESGPU_EINVAL
    empty = A.aesgpu_batch_plan(ctx, A.make_msgs([0], [0], [0], [0], [128], [0], [0]))
    assert A.aesgpu_batch_run(empty, None, 0, None, None, 0, 0) == A.AESGPU_OK
    A.aesgpu_batch_free(empty)


def test_full_batched_workload(A, ctx):
    """65,536 messages, 16 B .. 1 MiB log-uniform, seed 3: one encrypt run and
    one decrypt run of the random input, each compared in full with the
    oracle (the SHA-256 of the whole packed output equals the digest of the
    oracle's, from golden/full_size_digests.json); 2,000 random messages plus
    the 50 longest and 50 shortest are also recomputed by the oracle one by
    one, to name a wrong message; and the whole batch round-trips."""
    import hashlib

    import torch
    from gpu_common import full_size_digests, sha256_dev
    from paper_1201_0398_amd import workloads
    log("case: batched workload seed 3 (generating)")
    g = full_size_digests()
    w = workloads.batched(seed=3)
    m = w.lengths.size
    assert w.total_bytes == g["batched_total_bytes"]
    assert hashlib.sha256(memoryview(w.data)).hexdigest() == g["batched_input_sha256"], \
        "the batched input recipe changed"
    log(f"{m} messages, {w.total_bytes} bytes")
    zeros = np.zeros(m, dtype=np.int64)
    enc = A.make_msgs(w.offsets, w.offsets, w.lengths, np.arange(m), w.key_bits, w.modes, zeros,
                      w.nonces, w.ctr0)
    dec = A.make_msgs(w.offsets, w.offsets, w.lengths, np.arange(m), w.key_bits, w.modes,
                      zeros + 1, w.nonces, w.ctr0)
    pe, pd = A.aesgpu_batch_plan(ctx, enc), A.aesgpu_batch_plan(ctx, dec)
    try:
        d_keys = to_dev(w.keys.reshape(-1))
        d_in = to_dev(w.data)
        d_ct = torch.empty_like(d_in)
        A.aesgpu_batch_run(pe, d_keys, m, d_in, d_ct)
        order = np.argsort(w.lengths)
        rng = np.random.default_rng(3)
        pick = np.unique(np.concatenate([rng.choice(m, 2000, replace=False), order[:50],
                                         order[-50:]]))
        for j in pick:
            o, L = int(w.offsets[j]), int(w.lengths[j])
            key = w.keys[j, : w.key_bits[j] // 8]
            src = w.data[o:o + L]
            want = oracle.ctr(key, w.nonces[j], 1, src) if w.modes[j] else oracle.ecb(key, src)
            got = from_dev(d_ct[o:o + L])
            assert np.array_equal(got, want), f"message {j} (len {L}, mode {w.modes[j]})"
        assert sha256_dev(d_ct) == g["batched_encrypt_sha256"], "batched encryption output"
        log("case: batched workload, decryption of the random input")
        d_pt = torch.empty_like(d_in)
        A.aesgpu_batch_run(pd, d_keys, m, d_in, d_pt)
        assert sha256_dev(d_pt) == g["batched_decrypt_sha256"], "batched decryption output"
        A.aesgpu_batch_run(pd, d_keys, m, d_ct, d_pt)
        assert torch.equal(d_pt, d_in), "batch round trip failed"
    finally:
        A.aesgpu_batch_free(pe)
        A.aesgpu_batch_free(pd)
