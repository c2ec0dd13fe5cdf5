"""Launch-shape autotuner for the batched AES launch.

The batched kernel has two shape parameters: blocks per lane (ILP inside a
wave) and blocks per tile (the unit a wave pulls from the queue; small tiles
balance better, large tiles amortise the per-tile key expansion and queue
traffic).  ``tune_batch`` times every candidate shape on the caller's own
batch and buffers (each candidate is a real ``aesgpu_batch_run`` through the
C ABI, timed with HIP events on the stream it runs on), keeps the fastest, and
records the choice in a JSON cache keyed by the GPU architecture and a coarse
signature of the workload, so the next batch of the same kind skips the
search.  All encryption work happens in the library's kernels; this module
only chooses parameters.

Cache file: ``$AESGPU_TUNE_CACHE`` if set, else ``~/.cache/aesgpu_tune.json``.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass

DEFAULT_CANDIDATES = [(bpl, tile) for bpl in (1, 2, 4) for tile in (1024, 2048, 4096, 8192)]


def cache_path() -> str:
    return os.environ.get("AESGPU_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "aesgpu_tune.json"))


def workload_key(arch: str, lengths, modes, dirs) -> str:
    """Coarse signature: total bytes and mean message bytes as powers of two,
    and the share of blocks that need the inverse tables in tenths."""
    import numpy as np
    lengths = np.asarray(lengths, dtype=np.float64)
    total = float(lengths.sum())
    if total <= 0:
        return f"{arch}|empty"
    inverse = float(lengths[(np.asarray(modes) == 0) & (np.asarray(dirs) == 1)].sum()) / total
    return (f"{arch}|total2^{int(math.log2(total))}|mean2^{int(math.log2(total / lengths.size))}"
            f"|inv{int(round(inverse * 10))}")


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(entries: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


@dataclass
class Choice:
    blocks_per_lane: int
    tile_blocks: int
    ms: float | None          # measured time of the chosen shape (None: from cache)
    timings: dict             # "(bpl, tile)" -> ms for every candidate tried
    from_cache: bool


def gpu_arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def tune_batch(ctx, msgs, lengths, modes, dirs, d_keys, n_key_slots: int, d_in, d_out,
               candidates=None, reps: int = 3, use_cache: bool = True,
               path: str | None = None) -> Choice:
    """Picks (blocks per lane, tile blocks) for this batch and returns it.

    ``msgs`` is the ``aesgpu_msg`` array for ``aesgpu_batch_plan``; lengths,
    modes and dirs are the per-message values it was built from (for the
    cache key).  Each candidate runs once to warm up and ``reps`` times timed.
    """
    import torch

    from . import aesgpu as A
    key = workload_key(gpu_arch(), lengths, modes, dirs)
    cache = load_cache(path) if use_cache else {}
    if use_cache and key in cache:
        c = cache[key]
        return Choice(int(c["blocks_per_lane"]), int(c["tile_blocks"]), None,
                      c.get("timings", {}), True)
    timings = {}
    best = None
    for bpl, tile in (candidates or DEFAULT_CANDIDATES):
        plan = A.aesgpu_batch_plan(ctx, msgs, blocks_per_lane=bpl, tile_blocks=tile)
        try:
            A.aesgpu_batch_run(plan, d_keys, n_key_slots, d_in, d_out)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                A.aesgpu_batch_run(plan, d_keys, n_key_slots, d_in, d_out)
            b.record()
            b.synchronize()
            ms = a.elapsed_time(b) / reps
        finally:
            A.aesgpu_batch_free(plan)
        timings[f"({bpl}, {tile})"] = round(ms, 4)
        if best is None or ms < best[2]:
            best = (bpl, tile, ms)
    if use_cache:
        cache[key] = {"blocks_per_lane": best[0], "tile_blocks": best[1], "timings": timings}
        store_cache(cache, path)
    return Choice(best[0], best[1], best[2], timings, False)
