"""Shared helpers of the GPU parity tests (all results compared to the oracle
bit for bit: AES is integer work, so the tolerance is zero)."""
import sys

import numpy as np
import pytest


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # noqa: BLE001
        return False


requires_gpu = pytest.mark.skipif(not gpu_available(), reason="needs a GPU")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def from_dev(t) -> np.ndarray:
    return t.cpu().numpy()


def sample_indices(n_blocks: int, rng: np.random.Generator, n_random: int = 8192,
                   edge: int = 2048, boundaries=()) -> np.ndarray:
    """Block indices to compare at full size: both ends, random positions and
    the blocks around given boundaries (tile and grid-stride edges)."""
    parts = [np.arange(min(edge, n_blocks)), np.arange(max(0, n_blocks - edge), n_blocks),
             rng.integers(0, n_blocks, size=n_random)]
    for b in boundaries:
        parts.append(np.arange(max(0, b - 2), min(n_blocks, b + 2)))
    return np.unique(np.concatenate(parts)).astype(np.int64)


def gather_blocks(dev_u8, idx: np.ndarray) -> np.ndarray:
    import torch
    blocks = dev_u8.view(-1, 16)
    ix = torch.from_numpy(idx).to(dev_u8.device)
    return blocks.index_select(0, ix).cpu().numpy()


def copy_device(dst: int, src: int, n: int) -> None:
    """Synchronous device-to-device copy of n bytes between raw addresses,
    through the HIP runtime torch has already loaded."""
    import ctypes

    import torch  # noqa: F401  (loads the HIP runtime)
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    rc = hip.hipMemcpy(dst, src, n, 3)  # hipMemcpyDeviceToDevice
    assert rc == 0, f"hipMemcpy failed: {rc}"


def sha256_dev(t, chunk: int = 1 << 28) -> str:
    """SHA-256 of a device uint8 tensor's bytes, copied to the host in chunks."""
    import hashlib
    h = hashlib.sha256()
    n = t.numel()
    for o in range(0, n, chunk):
        h.update(memoryview(t[o:o + chunk].cpu().numpy()))
    return h.hexdigest()


def full_size_digests() -> dict:
    """Digests of the oracle's whole outputs on the full-size workloads,
    written by tests/golden/make_full_digests.py from the oracle alone."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "full_size_digests.json")
    with open(path) as f:
        return json.load(f)
