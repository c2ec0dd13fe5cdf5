"""GPU parity of CBC inside the batched launch: block-parallel CBC decryption
tiles and the CBC-encryption launch (four lanes per message, groups of up to 16
messages of one key size), mixed with ECB and CTR messages, against the CPU
oracle run on each message alone; in-place rules and plan validation."""
import numpy as np
import pytest

import oracle
from gpu_common import from_dev, full_size_digests, log, requires_gpu, sha256_dev, to_dev

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


def _batch(rng, m, modes, max_blocks=512):
    """m messages with the given modes (0 ECB, 1 CTR, 2 CBC), random
    directions, key sizes, lengths and gaps; CBC and ECB whole blocks."""
    blocks = rng.integers(1, max_blocks + 1, size=m)
    lengths = 16 * blocks
    tail = rng.integers(0, 16, size=m)
    lengths = np.where(modes == 1, np.maximum(lengths - tail, 1), lengths)
    bits = np.array([128, 192, 256])[rng.integers(0, 3, size=m)]
    dirs = rng.integers(0, 2, size=m)
    pad = 16 * rng.integers(0, 3, size=m)
    span = 16 * ((lengths + 15) // 16) + pad
    in_off = np.concatenate([[0], np.cumsum(span)[:-1]])
    out_off = np.concatenate([[0], np.cumsum(span[::-1])[:-1]])[::-1].copy()
    keys = np.zeros((m, 32), dtype=np.uint8)
    for j in range(m):
        keys[j, : bits[j] // 8] = rng.integers(0, 256, bits[j] // 8, dtype=np.uint8)
    nonces = rng.integers(0, 256, (m, 12), dtype=np.uint8)
    ctr0 = rng.integers(0, 1 << 31, size=m).astype(np.uint32)
    ivs = rng.integers(0, 256, (m, 16), dtype=np.uint8)
    total = int(span.sum())
    data = rng.integers(0, 256, total, dtype=np.uint8)
    return dict(lengths=lengths, modes=modes, bits=bits, dirs=dirs, in_off=in_off,
                out_off=out_off, keys=keys, nonces=nonces, ctr0=ctr0, ivs=ivs, data=data,
                total=total, m=m)


def _expected(b, j, data=None):
    data = b["data"] if data is None else data
    L = int(b["lengths"][j])
    key = b["keys"][j, : b["bits"][j] // 8]
    src = data[b["in_off"][j]: b["in_off"][j] + L]
    if b["modes"][j] == 1:
        return oracle.ctr(key, b["nonces"][j], int(b["ctr0"][j]), src)
    if b["modes"][j] == 2:
        if b["dirs"][j]:
            return oracle.cbc_decrypt(key, b["ivs"][j], src)
        return oracle.cbc_encrypt(key, b["ivs"][j], src)
    return oracle.ecb(key, src, decrypt=bool(b["dirs"][j]))


def _msgs(A, b, dirs=None):
    return A.make_msgs(b["in_off"], b["out_off"], b["lengths"], np.arange(b["m"]), b["bits"],
                       b["modes"], b["dirs"] if dirs is None else dirs, b["nonces"], b["ctr0"],
                       iv=b["ivs"])


def _run_and_check(A, ctx, b, **kw):
    import torch
    plan = A.aesgpu_batch_plan(ctx, _msgs(A, b), **kw)
    try:
        st = A.aesgpu_batch_info(plan)
        has_enc = bool(((b["modes"] == 2) & (b["dirs"] == 0)).any())
        has_block = bool(((b["modes"] != 2) | (b["dirs"] == 1)).any())
        assert st.launches == int(has_enc) + int(has_block)
        d_keys = to_dev(b["keys"].reshape(-1))
        d_in = to_dev(b["data"])
        d_out = torch.full((b["total"],), 0x5A, dtype=torch.uint8, device="cuda")
        for _ in range(2):    # a graph replay (or a second direct run) too
            A.aesgpu_batch_run(plan, d_keys, b["m"], d_in, d_out)
        out = from_dev(d_out)
        covered = np.zeros(b["total"], dtype=bool)
        for j in range(b["m"]):
            o, L = int(b["out_off"][j]), int(b["lengths"][j])
            assert np.array_equal(out[o:o + L], _expected(b, j)), \
                f"message {j}: mode {b['modes'][j]} dir {b['dirs'][j]} bits {b['bits'][j]} len {L}"
            covered[o:o + L] = True
        assert (out[~covered] == 0x5A).all(), "wrote outside the messages"
    finally:
        A.aesgpu_batch_free(plan)


@pytest.mark.parametrize("bpl,graph", [(1, True), (2, True), (2, False), (4, True)])
def test_mixed_batch_with_cbc(A, ctx, bpl, graph):
    rng = np.random.default_rng(9000 + bpl + 10 * graph)
    m = 600
    modes = rng.integers(0, 3, size=m)
    b = _batch(rng, m, modes)
    log(f"case: mixed ECB/CTR/CBC batch of {m}, bpl={bpl} graph={graph}, {b['total']} bytes")
    flags = 0 if graph else A.AESGPU_BATCH_NO_GRAPH
    _run_and_check(A, ctx, b, blocks_per_lane=bpl, tile_blocks=128 * bpl, flags=flags)


@pytest.mark.parametrize("bpl,tile", [(2, 256), (4, 512), (4, 8192)])
def test_ragged_tile_ends_every_mode(A, ctx, bpl, tile):
    """Message lengths at and around multiples of a step (64 blocks per lane
    slot times blocks per lane) and of the tile, in every mode and direction:
    the whole steps, the 64-block groups after them and the tile cuts must
    cover every block once."""
    rng = np.random.default_rng(9050 + bpl + tile)
    step = 64 * bpl
    counts = sorted({1, 63, 64, 65, step - 1, step, step + 1, 2 * step + 63, 3 * step + 64,
                     tile - 1, tile, tile + 1, tile + step - 1, 2 * tile + 65})
    kinds = [(0, 0, 0), (0, 1, 0), (2, 1, 0), (2, 0, 0), (1, 0, 0), (1, 0, 9)]  # mode, dir, CTR tail
    specs = [(c, k) for c in counts for k in kinds]
    m = len(specs)
    b = _batch(rng, m, np.array([k[0] for _, k in specs]), max_blocks=1)
    lengths = np.array([16 * c - (k[2] and 16 - k[2]) for c, k in specs])
    b["lengths"] = lengths
    b["dirs"] = np.array([k[1] for _, k in specs])
    span = 16 * ((lengths + 15) // 16) + 16
    b["in_off"] = np.concatenate([[0], np.cumsum(span)[:-1]])
    b["out_off"] = np.concatenate([[0], np.cumsum(span[::-1])[:-1]])[::-1].copy()
    b["total"] = int(span.sum())
    b["data"] = rng.integers(0, 256, b["total"], dtype=np.uint8)
    log(f"case: {m} messages around step {step} and tile {tile}, {b['total']} bytes")
    _run_and_check(A, ctx, b, blocks_per_lane=bpl, tile_blocks=tile)


@pytest.mark.parametrize("m", [1, 15, 16, 17, 65, 1000])
def test_cbc_only_batches(A, ctx, m):
    """Only CBC messages: encrypt groups of up to 16 per key size (full,
    partial and many groups), and decrypt tiles."""
    rng = np.random.default_rng(9100 + m)
    b = _batch(rng, m, np.full(m, 2), max_blocks=300)
    log(f"case: CBC-only batch of {m}")
    _run_and_check(A, ctx, b)
    b["dirs"][:] = 0                    # encrypt only: one launch
    _run_and_check(A, ctx, b)


def test_cbc_round_trip_and_in_place(A, ctx):
    import torch
    rng = np.random.default_rng(9200)
    m = 150
    b = _batch(rng, m, np.full(m, 2), max_blocks=700)
    b["out_off"] = b["in_off"].copy()                     # in place layout
    d_keys = to_dev(b["keys"].reshape(-1))
    buf = to_dev(b["data"])
    enc = A.aesgpu_batch_plan(ctx, _msgs(A, b, dirs=np.zeros(m, dtype=np.int64)))
    dec = A.aesgpu_batch_plan(ctx, _msgs(A, b, dirs=np.ones(m, dtype=np.int64)))
    try:
        A.aesgpu_batch_run(enc, d_keys, m, buf, buf)      # CBC encryption in place
        ct = from_dev(buf)
        bb = dict(b, dirs=np.zeros(m, dtype=np.int64))
        for j in range(m):
            o, L = int(b["in_off"][j]), int(b["lengths"][j])
            assert np.array_equal(ct[o:o + L], _expected(bb, j)), f"message {j}"
        # CBC decryption in place is refused; out of place it restores the data.
        st = A.aesgpu_batch_run(dec, d_keys, m, buf, buf, check=False)
        assert st == A.AESGPU_EINVAL
        out = torch.zeros_like(buf)
        A.aesgpu_batch_run(dec, d_keys, m, buf, out)
        pt = from_dev(out)
        for j in range(m):
            o, L = int(b["in_off"][j]), int(b["lengths"][j])
            assert np.array_equal(pt[o:o + L], b["data"][o:o + L]), f"message {j}"
    finally:
        A.aesgpu_batch_free(enc)
        A.aesgpu_batch_free(dec)


def test_cbc_encrypt_one_long_message_golden(A, ctx):
    """One 1 MiB message (65,536 sequential blocks) of the seed-0 workload
    through the CBC-encryption launch, against the stored oracle digest."""
    import hashlib
    import json
    import os

    import torch
    from paper_1201_0398_amd import workloads
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                          "oracle_digests.json")
    w = workloads.single_small(seed=0)
    n = w.data.size
    keys = np.zeros(32, dtype=np.uint8)
    keys[:16] = w.keys[128]
    msgs = A.make_msgs([0], [0], [n], [0], [128], [A.AESGPU_MODE_CBC], [0],
                       iv=np.asarray(w.iv).reshape(1, 16))
    plan = A.aesgpu_batch_plan(ctx, msgs)
    try:
        d_out = torch.empty(n, dtype=torch.uint8, device="cuda")
        A.aesgpu_batch_run(plan, to_dev(keys), 1, to_dev(w.data), d_out)
        got = hashlib.sha256(from_dev(d_out).tobytes()).hexdigest()
        assert got == json.load(open(golden))["cbc128_encrypt_sha256"]
    finally:
        A.aesgpu_batch_free(plan)


def test_full_cbc_batch_workload(A, ctx):
    """The 65,536-message CBC workload the benchmark times (seed 6): every
    output byte of the encryption launch and of the decryption launch (the same
    input taken as ciphertext) against digests of the oracle's outputs
    (``golden/full_size_digests.json``), plus the first 64 messages each
    recomputed by the oracle, to name a wrong message."""
    import hashlib

    import torch
    from paper_1201_0398_amd import workloads
    dg = full_size_digests()
    w = workloads.cbc_batch(seed=6)
    assert hashlib.sha256(memoryview(w.data)).hexdigest() == dg["cbc_batch_input_sha256"], \
        "the CBC batch input recipe changed"
    m = w.lengths.size
    d_keys = torch.from_numpy(w.keys.reshape(-1).copy()).to("cuda")
    d_in = to_dev(w.data)
    for name, direction in (("encrypt", 0), ("decrypt", 1)):
        log(f"case: 65,536-message CBC batch, {name}")
        msgs = A.make_msgs(w.offsets, w.offsets, w.lengths, np.arange(m), w.key_bits,
                           np.full(m, A.AESGPU_MODE_CBC), np.full(m, direction), iv=w.ivs)
        plan = A.aesgpu_batch_plan(ctx, msgs)
        try:
            d_out = torch.zeros_like(d_in)
            A.aesgpu_batch_run(plan, d_keys, m, d_in, d_out)
            torch.cuda.synchronize()
        finally:
            A.aesgpu_batch_free(plan)
        out = from_dev(d_out)
        f = oracle.cbc_encrypt if direction == 0 else oracle.cbc_decrypt
        for j in range(64):
            o, L = int(w.offsets[j]), int(w.lengths[j])
            key = w.keys[j, : int(w.key_bits[j]) // 8]
            assert np.array_equal(out[o:o + L], f(key, w.ivs[j], w.data[o:o + L])), f"message {j}"
        assert sha256_dev(d_out) == dg[f"cbc_batch_{name}_sha256"], f"CBC batch {name}"


def test_cbc_plan_validation(A, ctx):
    import ctypes
    msgs = A.make_msgs([0], [0], [24], [0], [128], [A.AESGPU_MODE_CBC], [0])
    out = ctypes.c_void_p()
    L = A.lib()
    assert L.aesgpu_batch_plan(ctx, msgs, 1, None, ctypes.byref(out)) == A.AESGPU_EINVAL
    msgs = A.make_msgs([0], [0], [32], [0], [128], [3], [0])
    assert L.aesgpu_batch_plan(ctx, msgs, 1, None, ctypes.byref(out)) == A.AESGPU_EINVAL
    # A zero-length CBC message is valid and does nothing.
    msgs = A.make_msgs([0, 0], [0, 16], [0, 16], [0, 0], [128, 128], [2, 2], [0, 0])
    plan = A.aesgpu_batch_plan(ctx, msgs)
    try:
        assert A.aesgpu_batch_info(plan).launches == 1
    finally:
        A.aesgpu_batch_free(plan)
