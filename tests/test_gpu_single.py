"""GPU parity of the single-buffer calls (ECB both ways, CTR, the paper's
LE-128 CTR, CBC decryption) against the CPU oracle, at sizes that span several
tiles and a ragged tail, plus the edge cases and argument errors; every test
runs with the blocks per lane chosen by size and with each of 1, 2 and 4
forced."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from gpu_common import from_dev, log, requires_gpu, to_dev

pytestmark = [pytest.mark.gpu, requires_gpu]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")
TILE = 1024 * 4          # blocks per workgroup step at 4 blocks per lane
# Sizes in blocks: tiny, wave and workgroup edges, tile edges, and one size that
# makes every workgroup of a 256-CU grid stride twice with a ragged end.
SIZES = [1, 2, 63, 64, 65, 1023, 1024, 1025, TILE - 1, TILE, TILE + 1, 3 * TILE + 77]
BIG = 2 * 256 * TILE + 4099


@pytest.fixture(scope="module")
def A():
    from paper_1201_0398_amd import aesgpu
    return aesgpu


@pytest.fixture(scope="module", params=[0, 1, 2, 4], ids=["bpl-auto", "bpl1", "bpl2", "bpl4"])
def ctx(A, request):
    """A context per blocks-per-lane setting: chosen by size (auto), or fixed
    to each kernel variant with AESGPU_FORCE_BPL (read at context creation),
    so that every test runs each variant."""
    import os
    old = os.environ.pop("AESGPU_FORCE_BPL", None)
    if request.param:
        os.environ["AESGPU_FORCE_BPL"] = str(request.param)
    try:
        c = A.aesgpu_create()
    finally:
        os.environ.pop("AESGPU_FORCE_BPL", None)
        if old is not None:
            os.environ["AESGPU_FORCE_BPL"] = old
    log(f"context with blocks per lane {request.param or 'chosen by size'}")
    yield c
    A.aesgpu_destroy(c)


def test_small_workload_ecb128(A, ctx):
    import torch
    from paper_1201_0398_amd import workloads
    log("case: 1 MiB ECB-128 seed 0")
    w = workloads.single_small(seed=0)
    key = w.keys[128]
    k = A.aesgpu_expand_key(key)
    d_in = to_dev(w.data)
    d_ct, d_pt = torch.empty_like(d_in), torch.empty_like(d_in)
    A.aesgpu_ecb_encrypt(ctx, k, d_in, d_ct)
    A.aesgpu_ecb_decrypt(ctx, k, d_ct, d_pt)
    A.aesgpu_ecb_decrypt(ctx, k, d_in, d_in)          # in place
    torch.cuda.synchronize()
    ct = from_dev(d_ct)
    assert np.array_equal(ct, oracle.ecb_encrypt(key, w.data))
    assert np.array_equal(from_dev(d_pt), w.data)
    assert np.array_equal(from_dev(d_in), oracle.ecb_decrypt(key, w.data))
    g = json.load(open(GOLDEN))
    assert hashlib.sha256(ct.tobytes()).hexdigest() == g["ecb128_encrypt_sha256"]


def test_small_workload_paper_modes(A, ctx):
    """The 1 MiB seed-0 workload through the paper's CTR counter and CBC
    decryption, against the stored oracle digests."""
    import torch
    from paper_1201_0398_amd import workloads
    log("case: 1 MiB LE-128 CTR and CBC decrypt seed 0")
    w = workloads.single_small(seed=0)
    key = w.keys[128]
    k = A.aesgpu_expand_key(key)
    g = json.load(open(GOLDEN))
    d_in = to_dev(w.data)
    d_out = torch.empty_like(d_in)
    A.aesgpu_ctr_le128_xcrypt(ctx, k, w.iv, 0, d_in, d_out)
    assert hashlib.sha256(from_dev(d_out).tobytes()).hexdigest() == g["ctr_le128_index0_0_sha256"]
    A.aesgpu_cbc_decrypt(ctx, k, w.iv, d_in, d_out)
    assert hashlib.sha256(from_dev(d_out).tobytes()).hexdigest() == \
        g["cbc128_decrypt_of_input_sha256"]


@pytest.mark.parametrize("kb", [16, 24, 32])
@pytest.mark.parametrize("decrypt", [False, True], ids=["enc", "dec"])
def test_ecb_sizes(A, ctx, kb, decrypt):
    import torch
    rng = np.random.default_rng(1000 + kb + decrypt)
    key = rng.integers(0, 256, kb, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    fn = A.aesgpu_ecb_decrypt if decrypt else A.aesgpu_ecb_encrypt
    for n in SIZES:
        log(f"case: ECB-{8 * kb} {'dec' if decrypt else 'enc'} n_blocks={n}")
        data = rng.integers(0, 256, 16 * n, dtype=np.uint8)
        d_in = to_dev(data)
        # Guard bytes after the output catch writes past the end.
        d_out = torch.full((16 * n + 64,), 0x5A, dtype=torch.uint8, device="cuda")
        fn(ctx, k, d_in, d_out, n)
        out = from_dev(d_out)
        assert np.array_equal(out[: 16 * n], oracle.ecb(key, data, decrypt)), f"n={n}"
        assert (out[16 * n:] == 0x5A).all(), "wrote past the end"


def test_ecb_grid_stride_ragged(A, ctx):
    import torch
    rng = np.random.default_rng(7)
    key = rng.integers(0, 256, 16, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    data = rng.integers(0, 256, 16 * BIG, dtype=np.uint8)
    log(f"case: ECB-128 enc/dec n_blocks={BIG}")
    d_in = to_dev(data)
    d_ct = torch.empty_like(d_in)
    A.aesgpu_ecb_encrypt(ctx, k, d_in, d_ct)
    ct = from_dev(d_ct)
    assert np.array_equal(ct, oracle.ecb_encrypt(key, data))
    A.aesgpu_ecb_decrypt(ctx, k, d_ct, d_ct)
    assert np.array_equal(from_dev(d_ct), data)


def test_zero_length_is_noop(A, ctx):
    import torch
    k = A.aesgpu_expand_key(bytes(16))
    d = torch.full((32,), 7, dtype=torch.uint8, device="cuda")
    A.aesgpu_ecb_encrypt(ctx, k, d, d, 0)
    A.aesgpu_ecb_decrypt(ctx, k, d, d, 0)
    A.aesgpu_ctr_xcrypt(ctx, k, bytes(12), 1, d, d, 0)
    A.aesgpu_cbc_decrypt(ctx, k, bytes(16), d[:16], d[16:], 0)
    torch.cuda.synchronize()
    assert (from_dev(d) == 7).all()


@pytest.mark.parametrize("kb", [16, 24, 32])
def test_ctr_lengths_and_counters(A, ctx, kb):
    import torch
    rng = np.random.default_rng(2000 + kb)
    key = rng.integers(0, 256, kb, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    for n_bytes in [1, 15, 16, 17, 1000, 16 * 1024 - 1, 16 * TILE + 9, 16 * (3 * TILE + 77) + 15]:
        n_blocks = (n_bytes + 15) // 16
        for ctr0 in [1, int(rng.integers(0, 1 << 31)), (1 << 32) - n_blocks]:
            log(f"case: CTR-{8 * kb} n_bytes={n_bytes} ctr0={ctr0}")
            nonce = rng.integers(0, 256, 12, dtype=np.uint8)
            data = rng.integers(0, 256, n_bytes, dtype=np.uint8)
            d_in = to_dev(data)
            d_out = torch.full((n_bytes + 64,), 0x5A, dtype=torch.uint8, device="cuda")
            A.aesgpu_ctr_xcrypt(ctx, k, nonce, ctr0, d_in, d_out, n_bytes)
            out = from_dev(d_out)
            assert np.array_equal(out[:n_bytes], oracle.ctr(key, nonce, ctr0, data))
            assert (out[n_bytes:] == 0x5A).all(), "wrote past the end"


@pytest.mark.parametrize("kb", [16, 32])
def test_ctr_counter_alignment_and_carries(A, ctx, kb):
    """Counters at every offset modulo 64 that the lane mapping shifts by, and
    runs that carry into bytes 1, 2 and 3 of the 32-bit counter mid-call."""
    import torch
    rng = np.random.default_rng(2500 + kb)
    key = rng.integers(0, 256, kb, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    n_bytes = 16 * (2 * TILE + 300) + 7
    n_blocks = (n_bytes + 15) // 16
    starts = [0, 63, 64, 65, 127, 0xFF - 40, 0xFFFF - 5000, 0xFFFFFF - 70000,
              (1 << 32) - n_blocks - 1]
    for ctr0 in starts:
        log(f"case: CTR-{8 * kb} n_bytes={n_bytes} ctr0={ctr0:#x}")
        nonce = rng.integers(0, 256, 12, dtype=np.uint8)
        data = rng.integers(0, 256, n_bytes, dtype=np.uint8)
        d_in = to_dev(data)
        d_out = torch.full((n_bytes + 64,), 0x5A, dtype=torch.uint8, device="cuda")
        A.aesgpu_ctr_xcrypt(ctx, k, nonce, ctr0, d_in, d_out, n_bytes)
        out = from_dev(d_out)
        assert np.array_equal(out[:n_bytes], oracle.ctr(key, nonce, ctr0, data))
        assert (out[n_bytes:] == 0x5A).all(), "wrote past the end"
    for n_bytes in [1, 16 * 63, 16 * 64 + 1, 16 * 65]:       # less than one wave
        for ctr0 in [0, 1, 62, 63]:
            nonce = rng.integers(0, 256, 12, dtype=np.uint8)
            data = rng.integers(0, 256, n_bytes, dtype=np.uint8)
            d_in = to_dev(data)
            d_out = torch.full((n_bytes + 64,), 0x5A, dtype=torch.uint8, device="cuda")
            A.aesgpu_ctr_xcrypt(ctx, k, nonce, ctr0, d_in, d_out, n_bytes)
            out = from_dev(d_out)
            assert np.array_equal(out[:n_bytes], oracle.ctr(key, nonce, ctr0, data)), (n_bytes, ctr0)
            assert (out[n_bytes:] == 0x5A).all(), "wrote past the end"


def test_ctr_involution_chunking_and_overflow(A, ctx):
    import torch
    rng = np.random.default_rng(3)
    key = rng.integers(0, 256, 32, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    nonce = rng.integers(0, 256, 12, dtype=np.uint8)
    data = rng.integers(0, 256, 16 * 10000 + 3, dtype=np.uint8)
    d_in = to_dev(data)
    d_a = torch.empty_like(d_in)
    A.aesgpu_ctr_xcrypt(ctx, k, nonce, 1, d_in, d_a)
    d_b = torch.empty_like(d_in)
    cut = 16 * 4321
    A.aesgpu_ctr_xcrypt(ctx, k, nonce, 1, d_in[:cut], d_b[:cut])
    A.aesgpu_ctr_xcrypt(ctx, k, nonce, 1 + 4321, d_in[cut:], d_b[cut:])
    assert torch.equal(d_a, d_b), "chunked CTR differs from one call"
    A.aesgpu_ctr_xcrypt(ctx, k, nonce, 1, d_a, d_a)          # in place, inverse
    assert torch.equal(d_a, d_in), "CTR is not its own inverse"
    st = A.aesgpu_ctr_xcrypt(ctx, k, nonce, (1 << 32) - 1, d_in[:32], d_b[:32], check=False)
    assert st == A.AESGPU_ECTR_OVERFLOW


@pytest.mark.parametrize("kb", [16, 32])
def test_ctr_le128_matches_oracle(A, ctx, kb):
    import torch
    rng = np.random.default_rng(4000 + kb)
    key = rng.integers(0, 256, kb, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    ivs = [rng.integers(0, 256, 16, dtype=np.uint8),
           np.frombuffer(((1 << 32) - 5).to_bytes(16, "little"), dtype=np.uint8),
           np.frombuffer(((1 << 64) - 7).to_bytes(16, "little"), dtype=np.uint8),
           np.frombuffer(((1 << 128) - 9).to_bytes(16, "little"), dtype=np.uint8)]
    for iv in ivs:
        for index0 in (0, (1 << 32) - 100):
            n_bytes = 16 * (TILE + 300) + 7
            log(f"case: CTR-LE128-{8 * kb} index0={index0}")
            data = rng.integers(0, 256, n_bytes, dtype=np.uint8)
            d_in = to_dev(data)
            d_out = torch.empty_like(d_in)
            A.aesgpu_ctr_le128_xcrypt(ctx, k, iv, index0, d_in, d_out)
            assert np.array_equal(from_dev(d_out), oracle.ctr_le128(key, iv, index0, data))


def test_ctr_le128_alignment_and_short(A, ctx):
    """Counter starts at every residue the lane mapping shifts by (IV + index0
    modulo 256), runs shorter than a wave's 256 counters, and a start 3 blocks
    below a carry out of every 32-bit word."""
    import torch
    rng = np.random.default_rng(4100)
    key = rng.integers(0, 256, 16, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    base = rng.integers(0, 256, 16, dtype=np.uint8)
    top = np.frombuffer(((1 << 128) - 3).to_bytes(16, "little"), dtype=np.uint8)
    for iv, index0 in [(base, 0), (base, 1), (base, 255), (base, 256 + 77), (top, 0), (top, 2)]:
        for n_bytes in [1, 16 * 63 + 5, 16 * 255, 16 * 257 + 1, 16 * (2 * TILE + 9)]:
            log(f"case: CTR-LE128 index0={index0} n_bytes={n_bytes}")
            data = rng.integers(0, 256, n_bytes, dtype=np.uint8)
            d_in = to_dev(data)
            d_out = torch.full((n_bytes + 64,), 0x5A, dtype=torch.uint8, device="cuda")
            A.aesgpu_ctr_le128_xcrypt(ctx, k, iv, index0, d_in, d_out, n_bytes)
            out = from_dev(d_out)
            assert np.array_equal(out[:n_bytes], oracle.ctr_le128(key, iv, index0, data))
            assert (out[n_bytes:] == 0x5A).all(), "wrote past the end"


@pytest.mark.parametrize("kb", [16, 24, 32])
def test_cbc_decrypt_matches_oracle(A, ctx, kb):
    import torch
    rng = np.random.default_rng(5000 + kb)
    key = rng.integers(0, 256, kb, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    for n in [1, 2, 65, TILE + 1, 3 * TILE + 77]:
        log(f"case: CBC-{8 * kb} dec n_blocks={n}")
        iv = rng.integers(0, 256, 16, dtype=np.uint8)
        data = rng.integers(0, 256, 16 * n, dtype=np.uint8)
        d_in = to_dev(data)
        d_out = torch.empty_like(d_in)
        A.aesgpu_cbc_decrypt(ctx, k, iv, d_in, d_out)
        assert np.array_equal(from_dev(d_out), oracle.cbc_decrypt(key, iv, data))
        pt = oracle.cbc_decrypt(key, iv, data)
        assert np.array_equal(oracle.cbc_encrypt(key, iv, pt), data)
    st = A.aesgpu_cbc_decrypt(ctx, k, iv, d_in, d_in, check=False)
    assert st == A.AESGPU_EINVAL, "in-place CBC decryption must be rejected"


def test_argument_errors(A, ctx):
    import torch
    k = A.aesgpu_expand_key(bytes(24))
    d = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    p = d.data_ptr()
    L = A
    assert L.aesgpu_ecb_encrypt(ctx, k, p + 1, p + 512, 4, check=False) == A.AESGPU_EALIGN
    assert L.aesgpu_ecb_encrypt(ctx, k, p, p + 520, 4, check=False) == A.AESGPU_EALIGN
    assert L.aesgpu_ecb_encrypt(ctx, k, p, p + 16, 4, check=False) == A.AESGPU_EINVAL
    assert L.aesgpu_ecb_decrypt(ctx, k, p + 48, p, 4, check=False) == A.AESGPU_EINVAL
    assert L.aesgpu_ecb_encrypt(ctx, k, None, p, 4, check=False) == A.AESGPU_EINVAL
    assert L.aesgpu_ctr_xcrypt(ctx, k, bytes(12), 0, p, p + 16, 32, check=False) == \
        A.AESGPU_EINVAL
    bad = A.aesgpu_key()
    bad.key_bits, bad.nr = 128, 12
    assert L.aesgpu_ecb_encrypt(ctx, bad, p, p, 4, check=False) == A.AESGPU_EINVAL
    torch.cuda.synchronize()
    assert (from_dev(d) == 0).all(), "a rejected call touched memory"


def test_binding_refuses_short_tensors(A, ctx):
    """The library takes plain pointers; the binding refuses a tensor
    shorter than the size a call names before anything is launched."""
    import torch
    k = A.aesgpu_expand_key(bytes(16))
    a = torch.zeros(256, dtype=torch.uint8, device="cuda")
    b = torch.zeros(256, dtype=torch.uint8, device="cuda")
    calls = [
        lambda: A.aesgpu_ecb_encrypt(ctx, k, a, b, 17),
        lambda: A.aesgpu_ecb_decrypt(ctx, k, a, b[:64], 16),
        lambda: A.aesgpu_ctr_xcrypt(ctx, k, bytes(12), 1, a, b, 257),
        lambda: A.aesgpu_ctr_le128_xcrypt(ctx, k, bytes(16), 0, a[:100], b, 101),
        lambda: A.aesgpu_cbc_decrypt(ctx, k, bytes(16), a, b, 20),
    ]
    for call in calls:
        with pytest.raises(ValueError):
            call()
    torch.cuda.synchronize()
    assert (from_dev(a) == 0).all() and (from_dev(b) == 0).all()


def test_side_stream(A, ctx):
    import torch
    rng = np.random.default_rng(9)
    key = rng.integers(0, 256, 16, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    data = rng.integers(0, 256, 16 * 50000, dtype=np.uint8)
    d_in = to_dev(data)
    d_out = torch.empty_like(d_in)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        A.aesgpu_ecb_encrypt(ctx, k, d_in, d_out, stream=s)
    s.synchronize()
    assert np.array_equal(from_dev(d_out), oracle.ecb_encrypt(key, data))


def test_threads_and_streams_share_one_context(A, ctx):
    """Four host threads, each with its own stream, key size and mode, issue
    calls on one context at the same time (the context is immutable after
    creation); every output matches the oracle."""
    import threading

    import torch
    rng = np.random.default_rng(10)
    jobs = []
    for t in range(4):
        kb = (16, 24, 32, 16)[t]
        key = rng.integers(0, 256, kb, dtype=np.uint8)
        data = rng.integers(0, 256, 16 * (20000 + 777 * t), dtype=np.uint8)
        nonce = rng.integers(0, 256, 12, dtype=np.uint8)
        jobs.append(dict(key=key, data=data, nonce=nonce, d_in=to_dev(data)))
    torch.cuda.synchronize()
    errors = []

    def work(t, job):
        try:
            s = torch.cuda.Stream()
            k = A.aesgpu_expand_key(job["key"])
            d_a = torch.empty_like(job["d_in"])
            d_b = torch.empty_like(job["d_in"])
            for _ in range(5):
                A.aesgpu_ecb_encrypt(ctx, k, job["d_in"], d_a, stream=s)
                A.aesgpu_ecb_decrypt(ctx, k, d_a, d_b, stream=s)
                A.aesgpu_ctr_xcrypt(ctx, k, job["nonce"], 7, d_b, d_b, stream=s)
            s.synchronize()
            job["enc"], job["ctr"] = from_dev(d_a), from_dev(d_b)
        except Exception as e:  # noqa: BLE001
            errors.append((t, e))

    threads = [threading.Thread(target=work, args=(t, j)) for t, j in enumerate(jobs)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for j in jobs:
        assert np.array_equal(j["enc"], oracle.ecb_encrypt(j["key"], j["data"]))
        assert np.array_equal(j["ctr"], oracle.ctr(j["key"], j["nonce"], 7, j["data"]))


def test_small_buffer_tiles_every_mode(A, ctx):
    """Buffers in the one-block-per-lane range, which the kernel cuts into
    tiles of 64..1024 blocks, one per CU: sizes whose tiles are 64, 128, 320
    and 1024 blocks with ragged ends, one whose tiles make the grid stride,
    and the top of the range; every mode against the oracle, guard bytes
    after each output untouched."""
    import torch
    n_cu = A.aesgpu_ctx_num_cus(ctx)
    rng = np.random.default_rng(6100)
    key = rng.integers(0, 256, 16, dtype=np.uint8)
    k = A.aesgpu_expand_key(key)
    sizes = [n_cu * 64 - 5, n_cu * 128 - 1, n_cu * 300 + 5, n_cu * 1024 - 7, n_cu * 1024 + 3,
             n_cu * 2048 - 1]
    for n in sizes:
        data = rng.integers(0, 256, 16 * n, dtype=np.uint8)
        d_in = to_dev(data)
        d_out = torch.full((16 * n + 64,), 0x5A, dtype=torch.uint8, device="cuda")
        iv = rng.integers(0, 256, 16, dtype=np.uint8)
        nonce = rng.integers(0, 256, 12, dtype=np.uint8)
        ctr0 = int(rng.integers(0, 1 << 30))
        cases = [
            ("ecb enc", lambda: A.aesgpu_ecb_encrypt(ctx, k, d_in, d_out, n),
             lambda: oracle.ecb_encrypt(key, data)),
            ("ecb dec", lambda: A.aesgpu_ecb_decrypt(ctx, k, d_in, d_out, n),
             lambda: oracle.ecb_decrypt(key, data)),
            ("ctr", lambda: A.aesgpu_ctr_xcrypt(ctx, k, nonce, ctr0, d_in, d_out, 16 * n - 3),
             lambda: oracle.ctr(key, nonce, ctr0, data[:16 * n - 3])),
            ("ctr le128", lambda: A.aesgpu_ctr_le128_xcrypt(ctx, k, iv, 77, d_in, d_out, 16 * n),
             lambda: oracle.ctr_le128(key, iv, 77, data)),
            ("cbc dec", lambda: A.aesgpu_cbc_decrypt(ctx, k, iv, d_in, d_out, n),
             lambda: oracle.cbc_decrypt(key, iv, data)),
        ]
        for name, run, want in cases:
            log(f"case: small-buffer tiles, {name}, n_blocks={n}")
            d_out.fill_(0x5A)
            run()
            w = want()
            out = from_dev(d_out)
            assert np.array_equal(out[:w.size], w), f"{name} n_blocks={n}"
            assert (out[w.size:] == 0x5A).all(), f"{name} n_blocks={n}: wrote past the end"
