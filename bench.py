"""Benchmark of the AES hot path on one MI355X.

One step = key expansion (host) + AES-128 ECB encryption + AES-128 ECB
decryption + AES-128 CTR over a 1 GiB device-resident buffer of seeded random
bytes.  ``value`` is payload GB/s over the step (3 GiB of payload per step,
10^9 bytes per GB).  The dominant kernel's HBM roofline is measured live with
HIP events on the launch stream; the CPU oracle is timed on a bounded sample
of the same workload on the host cores.

Warm-up: W untimed steps, extended until --min-warmup-s (default 0.3 s) of
back-to-back work has passed, since the GPU clock ramps up over tens of
milliseconds of sustained load; the timed steps follow with no other GPU work
in between.  The JSON line's "warmup" is W as asked for; "warmup_steps_run"
and "warmup_s_run" are the steps and seconds actually run.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --copy-calibration   (plain 1 GiB device copies, for
                                             scaling HBM byte counters)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AES-128 ECB/CTR GB/s at 1 GiB (% HBM roofline); batched GB/s; serve p50/p99"
HBM_PEAK_GBS = 8000.0
# LDS table reads per AES-128 block issued to the LDS by each kernel (CTR takes
# 15 of its 148 from the scalar cache), and the LDS read peak: 256 CUs x 32
# lanes per clock x 2.4 GHz.
LDS_READS_PER_BLOCK = {"ecb_encrypt": 160, "ecb_decrypt": 160, "ctr_xcrypt": 133}
LDS_PEAK_TREADS = 256 * 32 * 2.4e9 / 1e12
GIB = 1 << 30
SERVE_SOURCE_BYTES = 2 * GIB


HBM_SUMMARY = os.path.join(ROOT, "profiles", "aes128_1gib_hbm_bytes.md")
KERNEL_SOURCES = ["aes_kernels.hip", "aes_device.h", "aes_internal.h"]


def measured_traffic(kernel: str, n_bytes: int):
    """HBM bytes per launch from the committed rocprofv3 summary (FETCH_SIZE +
    WRITE_SIZE scaled by a plain copy), or None when the kernel sources have
    changed since the counters were taken or the workload size differs."""
    import hashlib
    if n_bytes != GIB or not os.path.exists(HBM_SUMMARY):
        return None
    h = hashlib.sha256(b"".join(
        open(os.path.join(ROOT, "paper_1201_0398_amd", "csrc", f), "rb").read()
        for f in KERNEL_SOURCES)).hexdigest()
    vals = {}
    for line in open(HBM_SUMMARY):
        if line.startswith("kernel_source_sha256:"):
            vals["sha"] = line.split(":", 1)[1].strip()
        elif line.startswith("traffic_bytes_per_launch"):
            name, v = line[len("traffic_bytes_per_launch"):].split(":")
            vals[name.strip()] = int(float(v))
    if vals.get("sha") != h:
        return None
    return vals.get(kernel)


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--min-warmup-s", type=float, default=0.3,
                    help="keep warming up until this much wall time has passed (the GPU "
                         "clock ramps up over tens of ms of sustained load)")
    ap.add_argument("--bytes", type=int, default=GIB)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-bytes", type=int, default=256 << 20)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-reps", type=int, default=5)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-pipeline", action="store_true")
    ap.add_argument("--no-cbc-batch", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=100000)
    ap.add_argument("--only-sizes", action="store_true",
                    help="time only AES-128 ECB encryption calls of 16 KiB..1 GiB (the per-call "
                         "floor of small buffers) and print them as one JSON line")
    return ap.parse_args()


def copy_calibration(torch, n_bytes: int, reps: int = 5) -> None:
    a = torch.randint(0, 256, (n_bytes,), dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {reps} copies of {n_bytes} bytes")


def warm_up(torch, fn, seconds: float) -> None:
    """Calls fn back to back for at least `seconds` (the GPU clock ramps up
    over tens of milliseconds of load)."""
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    while time.perf_counter() - t0 < seconds:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()


def time_call(torch, fn, reps: int) -> float:
    """Mean seconds per call, HIP events on the current stream."""
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) * 1e-3 / reps


def single_rates(torch, A, ctx, w, d_in, d_out, reps: int = 3) -> dict:
    """Single-buffer payload rates (bytes/s) per (key bits, mode) over d_in."""
    n = d_in.numel()
    rates = {}
    for bits in (128, 192, 256):
        k = A.aesgpu_expand_key(bytes(w.keys[bits]))
        rates[(bits, "ecb_enc")] = n / time_call(
            torch, lambda: A.aesgpu_ecb_encrypt(ctx, k, d_in, d_out), reps)
        rates[(bits, "ecb_dec")] = n / time_call(
            torch, lambda: A.aesgpu_ecb_decrypt(ctx, k, d_in, d_out), reps)
        rates[(bits, "ctr")] = n / time_call(
            torch, lambda: A.aesgpu_ctr_xcrypt(ctx, k, w.nonce, 1, d_in, d_out), reps)
        # The modes the paper adds: CBC decryption (Eq. (2)) and its CTR
        # flavour with a 128-bit little-endian counter (IV + block index).
        iv = bytes(w.nonce) + bytes(4)
        rates[(bits, "cbc_dec")] = n / time_call(
            torch, lambda: A.aesgpu_cbc_decrypt(ctx, k, iv, d_in, d_out), reps)
        rates[(bits, "ctr_le128")] = n / time_call(
            torch, lambda: A.aesgpu_ctr_le128_xcrypt(ctx, k, iv, 0, d_in, d_out), reps)
    return rates


def size_sweep(torch, A, ctx, w, d_in, d_out) -> list:
    """AES-128 ECB encryption of device-resident buffers from 16 KiB to 1 GiB:
    the per-call time where launch and staging dominate (small data, the
    regime the paper's section 3.1 discusses) up to the streaming rate.  Each
    size first runs for at least 20 ms untimed (the clock drops during runs
    of tiny calls) and is then timed over at least 20 ms of calls."""
    k = A.aesgpu_expand_key(bytes(w.keys[128]))
    rows = []
    for n in [1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22, 1 << 24, 1 << 26, 1 << 28, 1 << 30]:
        call = lambda: A.aesgpu_ecb_encrypt(ctx, k, d_in, d_out, n // 16)  # noqa: E731
        t_one = time_call(torch, call, 1)
        reps = max(5, int(0.02 / t_one) + 1)
        time_call(torch, call, reps)              # warm-up at this size
        t = time_call(torch, call, reps)
        rows.append({"bytes": n, "us": round(t * 1e6, 2), "GB_s": round(n / t / 1e9, 1)})
    return rows


def launch_floor(torch) -> dict:
    """The per-call floor of any kernel launched from Python back to back:
    torch's own elementwise add on a 16-byte tensor, timed like the AES calls."""
    tiny = torch.zeros(4, device="cuda")
    call = lambda: tiny.add_(1.0)  # noqa: E731
    time_call(torch, call, 2000)
    t = time_call(torch, call, 2000)
    return {"torch_add_16B_us": round(t * 1e6, 2),
            "what": "torch add_ on a 16-byte device tensor, back to back, HIP events"}


def batched_bench(torch, A, ctx, rates: dict, reps: int, warm_s: float) -> dict:
    """The 65,536-message batch (seed 3), encrypt direction, graph replays."""
    import numpy as np

    from paper_1201_0398_amd import workloads
    log("generating the batched workload (seed 3)")
    w = workloads.batched(seed=3)
    m = w.lengths.size
    msgs = A.make_msgs(w.offsets, w.offsets, w.lengths, np.arange(m), w.key_bits, w.modes,
                       np.zeros(m, dtype=np.int64), w.nonces, w.ctr0)
    d_keys = torch.from_numpy(w.keys.reshape(-1).copy()).to("cuda")
    d_in = torch.from_numpy(w.data.copy()).to("cuda")
    d_out = torch.empty_like(d_in)
    from paper_1201_0398_amd import autotune
    # Steady clock before the candidates are compared and the batch is timed.
    warm = A.aesgpu_batch_plan(ctx, msgs)
    warm_up(torch, lambda: A.aesgpu_batch_run(warm, d_keys, m, d_in, d_out), warm_s)
    A.aesgpu_batch_free(warm)
    log("autotuning the batch launch shape")
    choice = autotune.tune_batch(ctx, msgs, w.lengths, w.modes, np.zeros(m, dtype=np.int64),
                                 d_keys, m, d_in, d_out, reps=2, use_cache=False)
    plan = A.aesgpu_batch_plan(ctx, msgs, blocks_per_lane=choice.blocks_per_lane,
                               tile_blocks=choice.tile_blocks)
    info = A.aesgpu_batch_info(plan)
    log(f"timing the batch: {m} messages, {w.total_bytes} bytes")
    run = lambda: A.aesgpu_batch_run(plan, d_keys, m, d_in, d_out)  # noqa: E731
    warm_up(torch, run, warm_s)
    sec = time_call(torch, run, reps)
    # Reference time: every message at the single-buffer rate of its key size and mode.
    t_ref = sum(float(w.lengths[(w.key_bits == bits) & (w.modes == mode)].sum()) /
                rates[(bits, "ctr" if mode else "ecb_enc")]
                for bits in (128, 192, 256) for mode in (0, 1))
    t_128 = w.total_bytes / rates[(128, "ecb_enc")]
    A.aesgpu_batch_free(plan)
    return {"GB_s": round(w.total_bytes / sec / 1e9, 1), "ms": round(sec * 1e3, 3),
            "messages": m, "bytes": int(w.total_bytes),
            "tiles": int(info.n_tiles_forward + info.n_tiles_inverse),
            "tile_blocks": int(info.tile_blocks), "blocks_per_lane": int(info.blocks_per_lane),
            "autotune_ms": choice.timings,
            "time_vs_single_buffer_mix": round(sec / t_ref, 3),
            "time_vs_single_buffer_aes128_ecb": round(sec / t_128, 3),
            "workload": "65,536 messages, log-uniform 16 B..1 MiB, own key each, key size "
                        "uniform over 128/192/256, ECB or CTR 50/50, encrypt, seed 3; one "
                        "persistent launch with device key expansion, hipGraph replay"}


def serving_bench(torch, A, ctx, n_requests: int, rates: dict | None = None, flags: int = 0,
                  at_rates: list | None = None) -> dict:
    """Poisson arrivals of ECB requests (64 B..16 MiB log-uniform, half encrypt,
    half decrypt, keys from a resident pool of 1,024), replayed natively
    against the continuous-batching server at fractions of its measured
    saturation rate (or at the request rates `at_rates`, to compare two
    server modes at equal load).  With the single-buffer rates, the
    saturation time is also compared with every request at the 1 GiB
    single-buffer rate of its key size and direction."""
    import numpy as np

    from paper_1201_0398_amd import workloads
    # Outputs stay in the arena from admission until the caller releases
    # them: near saturation (~0.8 TB/s, millisecond latencies) that is a few
    # GB, so a 4 GiB arena fills and starves admission; 16 GiB is under 6%
    # of the device memory.
    arena = 16 << 30
    # Request inputs are slices of a 2 GiB device-resident source pool, eight
    # times the 256 MB Infinity Cache, so that they stream from HBM as the
    # single-buffer runs they are compared with do.
    tr = workloads.serving(rate_per_s=1.0, n_requests=n_requests, seed=4,
                           source_bytes=SERVE_SOURCE_BYTES)
    std_gaps = np.diff(np.concatenate([[0.0], tr.arrivals]))  # Exp(1) gaps: scale per rate
    total = int(tr.sizes.sum())
    src = torch.from_numpy(tr.source.copy()).to("cuda")
    ptrs = src.data_ptr() + tr.src_offsets
    server = A.aesgpu_server_create(ctx, tr.pool_keys, tr.pool_bits, arena_bytes=arena,
                                    flags=flags)

    def replay(arrivals):
        reqs = A.make_requests(arrivals, ptrs, tr.sizes, tr.key_ids, tr.dirs)
        t0 = A.aesgpu_server_now(server) + 0.002
        done = A.aesgpu_server_replay(server, reqs, t0)
        t = np.array([(d.t_arrival, d.t_done) for d in done])
        lat = t[:, 1] - t[:, 0]
        span = t[:, 1].max() - t0
        return lat, span

    replay(np.zeros(n_requests))  # warm-up
    lat, span = replay(np.zeros(n_requests))
    lam_sat = n_requests / span
    points = []
    fracs = (0.1, 0.25, 0.5, 0.7, 0.85, 0.95)
    for i, frac in enumerate(fracs):
        lam = at_rates[i] if at_rates else frac * lam_sat
        frac = lam / lam_sat
        # Three replays per point: the median of each figure, and the worst
        # replay's p99 and lowest throughput beside it.
        p50, p99, gbs = [], [], []
        for _ in range(3):
            lat, span = replay(np.cumsum(std_gaps / lam))
            p50.append(float(np.median(lat)) * 1e6)
            p99.append(float(np.quantile(lat, 0.99)) * 1e6)
            gbs.append(total / span / 1e9)
        points.append({"frac_of_saturation": round(frac, 3), "rate_req_s": round(lam, 1),
                       "p50_us": round(float(np.median(p50)), 1),
                       "p99_us": round(float(np.median(p99)), 1),
                       "GB_s": round(float(np.median(gbs)), 1),
                       "p99_us_worst": round(max(p99), 1), "GB_s_lowest": round(min(gbs), 1)})
        log(f"serving at {frac:.2f} of saturation: {points[-1]} "
            f"(replays: p50 {[round(x) for x in p50]}, p99 {[round(x) for x in p99]})")
    st = A.aesgpu_server_get_stats(server)
    A.aesgpu_server_destroy(server)
    extra = {}
    if rates:
        bits = tr.pool_bits[tr.key_ids]
        t_ref = sum(float(tr.sizes[(bits == b) & (tr.dirs == d)].sum()) /
                    rates[(b, "ecb_dec" if d else "ecb_enc")]
                    for b in (128, 192, 256) for d in (0, 1))
        extra["saturation_time_vs_single_buffer_mix"] = round((n_requests / lam_sat) / t_ref, 3)
    return {**extra, "saturation_GB_s": round(total / (n_requests / lam_sat) / 1e9, 1),
            "saturation_req_s": round(lam_sat, 1), "requests_per_point": n_requests,
            "mean_request_bytes": round(total / n_requests, 1), "arena_bytes": arena,
            "source_pool_bytes": SERVE_SOURCE_BYTES,
            "batches": int(st.batches), "points": points,
            "workload": "Poisson arrivals, ECB requests 64 B..16 MiB log-uniform, 50/50 "
                        "encrypt/decrypt, 1,024 resident keys of mixed size, seed 4; inputs "
                        "device-resident slices of a 2 GiB pool; latency = completion seen by the host - arrival; "
                        "each point: median over three replays, with the worst p99 and "
                        "lowest GB/s of the three"}


def cbc_batch_bench(torch, A, ctx, reps: int, warm_s: float) -> dict:
    """65,536 short CBC messages (16 B..16 KiB, own key each, mixed key sizes,
    seed 6): the batched CBC-encryption launch (one message per lane,
    sequential within a message) and the block-parallel CBC decryption."""
    import numpy as np

    from paper_1201_0398_amd import workloads
    log("generating the CBC batch (seed 6)")
    w = workloads.cbc_batch(seed=6)
    m = w.lengths.size
    d_keys = torch.from_numpy(w.keys.reshape(-1).copy()).to("cuda")
    d_pt = torch.from_numpy(w.data.copy()).to("cuda")
    d_ct = torch.empty_like(d_pt)
    d_back = torch.empty_like(d_pt)
    out = {"workload": "65,536 CBC messages, log-uniform 16 B..16 KiB, own key and IV each, "
                       "key size uniform over 128/192/256, seed 6",
           "messages": m, "bytes": w.total_bytes}
    for name, direction, src, dst in (("encrypt", 0, d_pt, d_ct), ("decrypt", 1, d_ct, d_back)):
        msgs = A.make_msgs(w.offsets, w.offsets, w.lengths, np.arange(m), w.key_bits,
                           np.full(m, A.AESGPU_MODE_CBC), np.full(m, direction), iv=w.ivs)
        plan = A.aesgpu_batch_plan(ctx, msgs)
        try:
            run = lambda: A.aesgpu_batch_run(plan, d_keys, m, src, dst)  # noqa: E731
            warm_up(torch, run, warm_s)
            sec = time_call(torch, run, reps)
        finally:
            A.aesgpu_batch_free(plan)
        out[f"{name}_GB_s"] = round(w.total_bytes / sec / 1e9, 1)
        out[f"{name}_ms"] = round(sec * 1e3, 3)
    if not torch.equal(d_back, d_pt):
        raise SystemExit("CBC batch round trip failed")
    # Encryption is one block after another per message: the makespan over
    # the longest message's block count is the time per sequential block.
    out["encrypt_us_per_sequential_block"] = round(
        out["encrypt_ms"] * 1e3 / (int(w.lengths.max()) // 16), 3)
    return out


def pipeline_bench(torch, A, ctx, key_bytes: bytes) -> dict:
    """Host buffers in and out (the paper's upload / draw / read-back path):
    AES-128 ECB encryption through the chunked host-staged pipeline, wall time
    per call including both PCIe transfers, for pinned and pageable buffers
    over a range of sizes, with the kernel on host memory or with DMA copies;
    the plain pinned copy rates in each direction give the link's own bound."""
    import numpy as np
    k = A.aesgpu_expand_key(key_bytes)
    op = A.make_host_op(A.AESGPU_OP_ECB_ENCRYPT)
    top = 1 << 30
    a_in, h_in = A.aesgpu_host_alloc(top)
    a_out, h_out = A.aesgpu_host_alloc(top)
    rng = np.random.default_rng(5)
    h_in[:] = np.frombuffer(rng.bytes(top), dtype=np.uint8)
    out = {"op": "AES-128 ECB encrypt, host buffer in and out", "chunk_bytes": 8 << 20,
           "slots": 3}
    try:
        pl = A.aesgpu_pipeline_create(ctx, 8 << 20, 3)
        pl_dma = A.aesgpu_pipeline_create(ctx, 8 << 20, 3, A.AESGPU_PIPELINE_COPY)

        def wall(fn, n_bytes):
            reps = max(3, min(200, (256 << 20) // n_bytes))
            fn()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                fn()
                ts.append(time.perf_counter() - t0)
            return float(np.median(ts))

        for name, p in (("pinned_zero_copy", pl), ("pinned_dma_chunks", pl_dma)):
            rows = []
            for n in [1 << 16, 1 << 18, 1 << 20, 1 << 22, 1 << 24, 1 << 26, 1 << 28, 1 << 30]:
                t = wall(lambda: A.aesgpu_pipeline_run(p, k, op, a_in, a_out, n), n)
                rows.append({"bytes": n, "us": round(t * 1e6, 1), "GB_s": round(n / t / 1e9, 2)})
                log(f"pipeline {name} {n} B: {rows[-1]}")
            out[name] = rows
        # Pageable buffers: staged through the pipeline's pinned buffers, which
        # the kernel reads and writes (default) or which DMA copies move.
        src = np.asarray(h_in).copy()
        dst = np.empty_like(src)
        for name, p in (("pageable_staged", pl), ("pageable_dma_chunks", pl_dma)):
            rows = []
            for n in [1 << 20, 1 << 24, 1 << 28, 1 << 30]:
                t = wall(lambda: A.aesgpu_pipeline_run(p, k, op, src, dst, n), n)
                rows.append({"bytes": n, "us": round(t * 1e6, 1), "GB_s": round(n / t / 1e9, 2)})
                log(f"pipeline {name} {n} B: {rows[-1]}")
            out[name] = rows
        out["pageable_1GiB_GB_s"] = out["pageable_staged"][-1]["GB_s"]
        del src, dst
        A.aesgpu_pipeline_destroy(pl_dma)
        A.aesgpu_pipeline_destroy(pl)
        # The link alone: pinned 1 GiB copies each way (torch's own copies).
        dev = torch.empty(top, dtype=torch.uint8, device="cuda")
        hb = torch.empty(top, dtype=torch.uint8, pin_memory=True)
        t_h2d = wall(lambda: (dev.copy_(hb, non_blocking=True), torch.cuda.synchronize()), top)
        t_d2h = wall(lambda: (hb.copy_(dev, non_blocking=True), torch.cuda.synchronize()), top)
        out["pcie_h2d_GB_s"] = round(top / t_h2d / 1e9, 2)
        out["pcie_d2h_GB_s"] = round(top / t_d2h / 1e9, 2)
        del dev, hb
    finally:
        A.aesgpu_host_free(a_in)
        A.aesgpu_host_free(a_out)
    return out


def host_cores() -> dict:
    """The host CPU as this process sees it: cores online, cores it may run
    on, the CPU share the machine grants one GPU's jobs (its OMP_NUM_THREADS,
    where set) and the model name."""
    nproc = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = nproc
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or affinity
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         "")
    except OSError:
        pass
    return {"nproc": nproc, "affinity": affinity, "share": min(share, affinity), "model": model}


def cpu_baseline(sample_bytes: int) -> dict:
    """The oracle on every core of this process's CPU share: the host's
    OMP_NUM_THREADS where the machine sets it (its share of host cores per
    GPU), else every core the process may run on."""
    import numpy as np

    import oracle
    from paper_1201_0398_amd import workloads
    host = host_cores()
    threads = host["share"]
    w = workloads.single_1gib(seed=1, n_bytes=sample_bytes)
    key = w.keys[128]
    t0 = time.perf_counter()
    ct = oracle.ecb_encrypt(key, w.data, threads=threads)
    pt = oracle.ecb_decrypt(key, ct, threads=threads)
    ks = oracle.ctr(key, w.nonce, w.ctr0, w.data, threads=threads)
    dt = time.perf_counter() - t0
    assert np.array_equal(pt, w.data) and ks.size == w.data.size
    # One core, as the paper compares (section 3.1): the literal oracle, and
    # the oracle's own T-table path (the same algorithm as the GPU's, as the
    # paper's CPU implementation was), AES-128 ECB encryption.
    n1, nt = 1 << 20, 16 << 20
    t1 = time.perf_counter()
    oracle.ecb_encrypt(key, w.data[:n1], threads=1)
    t1 = time.perf_counter() - t1
    tt = time.perf_counter()
    oracle.ttable_ecb(key, w.data[:nt])
    tt = time.perf_counter() - tt
    return {"value": round(3 * sample_bytes / dt / 1e9, 6), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"AES-128 ECB enc+dec+CTR of the first {sample_bytes >> 20} MiB of the "
                      f"1 GiB seed-1 buffer, literal oracle, {threads} threads, {dt:.1f} s",
            "one_core_literal_GB_s": round(n1 / t1 / 1e9, 6),
            "one_core_ttable_GB_s": round(nt / tt / 1e9, 6),
            "host_nproc": host["nproc"], "host_affinity_cores": host["affinity"],
            "host_cpu": host["model"][:100],
            "cores_note": "threads = the host's OMP_NUM_THREADS (its CPU share per GPU) or "
                          "every core this process may run on"}


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the AES path "
              f"shards without communication, and this benchmark measures one GPU's share.",
              file=sys.stderr)
        return 2
    import numpy as np
    import torch

    if args.copy_calibration:
        copy_calibration(torch, args.bytes)
        return 0
    if args.only_sizes:
        from paper_1201_0398_amd import aesgpu as A
        from paper_1201_0398_amd import workloads
        w = workloads.single_1gib(seed=1, n_bytes=args.bytes)
        d_in = torch.from_numpy(w.data).to("cuda")
        d_out = torch.empty_like(d_in)
        ctx = A.aesgpu_create()
        rows = size_sweep(torch, A, ctx, w, d_in, d_out)
        A.aesgpu_destroy(ctx)
        print(json.dumps({"single_buffer_sizes_aes128_ecb_enc": rows,
                          "launch_floor": launch_floor(torch)}), flush=True)
        return 0

    from paper_1201_0398_amd import aesgpu as A
    from paper_1201_0398_amd import workloads

    n_bytes = args.bytes
    log(f"generating {n_bytes} bytes (seed 1)")
    w = workloads.single_1gib(seed=1, n_bytes=n_bytes)
    key = bytes(w.keys[128])
    d_in = torch.from_numpy(w.data).to("cuda")
    d_ct = torch.empty_like(d_in)
    d_pt = torch.empty_like(d_in)
    d_ctr = torch.empty_like(d_in)
    ctx = A.aesgpu_create()
    n_blocks = n_bytes // 16
    stream = torch.cuda.current_stream()
    names = ["ecb_encrypt", "ecb_decrypt", "ctr_xcrypt"]
    events = {n: [] for n in names}

    def step(record: bool):
        k = A.aesgpu_expand_key(key)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if record else None
        if record:
            ev[0].record(stream)
        A.aesgpu_ecb_encrypt(ctx, k, d_in, d_ct, n_blocks)
        if record:
            ev[1].record(stream)
        A.aesgpu_ecb_decrypt(ctx, k, d_ct, d_pt, n_blocks)
        if record:
            ev[2].record(stream)
        A.aesgpu_ctr_xcrypt(ctx, k, w.nonce, w.ctr0, d_in, d_ctr, n_bytes)
        if record:
            ev[3].record(stream)
            for i, n in enumerate(names):
                events[n].append((ev[i], ev[i + 1]))

    step(False)
    torch.cuda.synchronize()
    if not torch.equal(d_pt, d_in):
        raise SystemExit("round trip failed before timing")
    # Warm-up runs straight into the timed region (no other GPU work between),
    # W steps or longer, until min_warmup_s of back-to-back work has passed.
    warm, t_w = 0, time.perf_counter()
    while warm < args.warmup or time.perf_counter() - t_w < args.min_warmup_s:
        step(False)
        warm += 1
        if warm % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    warm_s = time.perf_counter() - t_w
    log(f"warmed up with {warm} steps ({args.warmup} asked for) in {warm_s:.2f} s; "
        f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    value = 3 * n_bytes / (dt / args.steps) / 1e9
    kern_ms = {n: float(np.mean([a.elapsed_time(b) for a, b in events[n]])) for n in names}
    dominant = max(kern_ms, key=kern_ms.get)
    algo_bytes = 2 * n_bytes  # read + write of the payload per launch
    achieved = algo_bytes / (kern_ms[dominant] * 1e-3) / 1e9
    per_kernel = {n: {"ms": round(kern_ms[n], 4),
                      "GB_s_payload": round(n_bytes / (kern_ms[n] * 1e-3) / 1e9, 1),
                      "hbm_frac": round(2 * n_bytes / (kern_ms[n] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
                  for n in names}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "warmup_steps_run": warm,
        "warmup_s_run": round(warm_s, 3), "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "AES-128 ECB encrypt + ECB decrypt + CTR (nonce||BE32, ctr0=1) of "
                               f"a {n_bytes >> 20} MiB uniform random device buffer, seed 1",
                   "payload_bytes_per_step": 3 * n_bytes},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dominant, n_bytes),
                     "algorithmic_bytes": algo_bytes,
                     "note": "32 B of HBM per 16-B block; the kernel is bound by LDS table-read "
                             "issue (160 random reads per AES-128 block, 2 LDS cycles per wave64 "
                             "read), see lds_roofline and "
                             "profiles/aes128_1gib_lds_valu_counters.md"},
        # The bound the kernel actually meets: LDS table reads, 32 lanes per
        # clock per CU (a wave64 ds_read_b32 takes 2 cycles) at 256 CUs and the
        # 2.4 GHz peak engine clock; 16 reads per round (paper section 2.1).
        "lds_roofline": {"bound": "lds", "kernel": dominant,
                         "achieved": round(LDS_READS_PER_BLOCK[dominant] * n_blocks /
                                           (kern_ms[dominant] * 1e-3) / 1e12, 3),
                         "peak": LDS_PEAK_TREADS, "unit": "T table reads/s",
                         "frac": round(LDS_READS_PER_BLOCK[dominant] * n_blocks /
                                       (kern_ms[dominant] * 1e-3) / 1e12 / LDS_PEAK_TREADS, 4),
                         "reads_per_block": LDS_READS_PER_BLOCK[dominant]},
        "kernels": per_kernel,
    }
    # The achievable HBM ceiling on this GPU: a plain device copy of the same
    # size (torch's copy kernel), read + write bytes over its event time.
    copy = lambda: d_pt.copy_(d_in)  # noqa: E731
    warm_up(torch, copy, 0.1)
    t_copy = time_call(torch, copy, 20)
    copy_gbs = 2 * n_bytes / t_copy / 1e9
    out["copy_ceiling"] = {"copy_GB_s": round(copy_gbs, 1), "unit": "GB/s (read + write)",
                           "dominant_kernel_frac_of_copy": round(achieved / copy_gbs, 4),
                           "copy_frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4),
                           "what": f"device-to-device copy of {n_bytes >> 20} MiB"}
    if not args.no_batched:
        rates = single_rates(torch, A, ctx, w, d_in, d_ct)
        out["single_buffer_GB_s"] = {f"aes{b}_{m}": round(v / 1e9, 1) for (b, m), v in rates.items()}
        out["single_buffer_sizes_aes128_ecb_enc"] = size_sweep(torch, A, ctx, w, d_in, d_ct)
        out["launch_floor"] = launch_floor(torch)
        del d_pt, d_ctr
        out["batched"] = batched_bench(torch, A, ctx, rates, args.batched_reps, args.min_warmup_s)
    if not args.no_serving:
        out["serving"] = serving_bench(torch, A, ctx, args.serve_requests,
                                       None if args.no_batched else rates)
        # The resident kernel at the same request rates, then its own saturation.
        out["serving_resident"] = serving_bench(
            torch, A, ctx, args.serve_requests, None if args.no_batched else rates,
            flags=A.AESGPU_SERVER_RESIDENT,
            at_rates=[p["rate_req_s"] for p in out["serving"]["points"]])
        out["serving_resident"]["mode"] = (
            "one resident kernel fed from rings in pinned host memory, at the same request "
            "rates as the batched server's points; frac_of_saturation is against the resident "
            "kernel's own saturation")
    if not args.no_cbc_batch:
        out["batched_cbc"] = cbc_batch_bench(torch, A, ctx, args.batched_reps, args.min_warmup_s)
    if not args.no_pipeline:
        out["host_pipeline"] = pipeline_bench(torch, A, ctx, key)
    A.aesgpu_destroy(ctx)
    del d_in, d_ct
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_bytes)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
