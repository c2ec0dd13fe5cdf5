"""ctypes binding of ``libaesgpu.so`` (C ABI declared in ``include/aesgpu.h``).

Functions keep the C names and only marshal arguments: device buffers are
torch tensors on a HIP device (or raw integer device addresses), streams are
torch streams (or raw ``hipStream_t`` integers; default: torch's current
stream).  Every byte of encryption runs in the library's HIP kernels; there is
no CPU path.  Loading fails loudly when the library has not been built.

torch is imported before the library is loaded so that the process holds one
HIP runtime: the library's dependency on ``libamdhip64.so.7`` then resolves
to the copy torch already loaded.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede loading the HIP library)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libaesgpu.so")

AESGPU_OK = 0
AESGPU_EINVAL = -1
AESGPU_EKEYLEN = -2
AESGPU_EALIGN = -3
AESGPU_ECTR_OVERFLOW = -4
AESGPU_ENOMEM = -5
AESGPU_EHIP = -6
AESGPU_EAGAIN = -7
AESGPU_ESCRATCH = -8
AESGPU_NOALLOC_SCRATCH_BYTES = 8 << 20


class AesgpuError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = _lib.aesgpu_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})")
        self.status = status


class aesgpu_key(ctypes.Structure):
    _fields_ = [("key_bits", ctypes.c_uint32), ("nr", ctypes.c_uint32),
                ("enc", ctypes.c_uint32 * 60), ("dec", ctypes.c_uint32 * 60)]


AESGPU_MODE_ECB = 0
AESGPU_MODE_CTR = 1
AESGPU_MODE_CBC = 2
AESGPU_DIR_ENCRYPT = 0
AESGPU_DIR_DECRYPT = 1
AESGPU_BATCH_NO_GRAPH = 1
AESGPU_SERVER_NO_DIRECT = 0xFFFFFFFF
AESGPU_SERVER_RESIDENT = 1


class aesgpu_msg(ctypes.Structure):
    _fields_ = [("in_off", ctypes.c_uint64), ("out_off", ctypes.c_uint64),
                ("n_bytes", ctypes.c_uint64), ("key_slot", ctypes.c_uint32),
                ("key_bits", ctypes.c_uint16), ("mode", ctypes.c_uint8), ("dir", ctypes.c_uint8),
                ("nonce", ctypes.c_uint8 * 12), ("ctr0", ctypes.c_uint32)]


class aesgpu_batch_config(ctypes.Structure):
    _fields_ = [("blocks_per_lane", ctypes.c_uint32), ("tile_blocks", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class aesgpu_batch_stats(ctypes.Structure):
    _fields_ = [("n_msgs", ctypes.c_uint64), ("n_tiles_forward", ctypes.c_uint64),
                ("n_tiles_inverse", ctypes.c_uint64), ("total_bytes", ctypes.c_uint64),
                ("in_bytes_needed", ctypes.c_uint64), ("out_bytes_needed", ctypes.c_uint64),
                ("blocks_per_lane", ctypes.c_uint32), ("tile_blocks", ctypes.c_uint32),
                ("launches", ctypes.c_uint32)]


class aesgpu_server_config(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("n_streams", ctypes.c_uint32),
                ("blocks_per_lane", ctypes.c_uint32), ("tile_blocks", ctypes.c_uint32),
                ("max_batch_requests", ctypes.c_uint32), ("max_batch_bytes", ctypes.c_uint64),
                ("max_queued", ctypes.c_uint32), ("direct_requests", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class aesgpu_done(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_uint32), ("d_out", ctypes.c_void_p),
                ("n_bytes", ctypes.c_uint64), ("t_arrival", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class aesgpu_request(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("t_arrival", ctypes.c_double),
                ("d_in", ctypes.c_void_p), ("n_bytes", ctypes.c_uint64),
                ("key_id", ctypes.c_uint32), ("dir", ctypes.c_uint32)]


AESGPU_OP_ECB_ENCRYPT = 0
AESGPU_OP_ECB_DECRYPT = 1
AESGPU_OP_CTR = 2
AESGPU_OP_CTR_LE128 = 3
AESGPU_OP_CBC_DECRYPT = 4


class aesgpu_host_op(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("ctr0", ctypes.c_uint32),
                ("nonce", ctypes.c_uint8 * 12), ("iv", ctypes.c_uint8 * 16)]


class aesgpu_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("batches", "requests_submitted", "requests_done", "bytes_done",
                 "max_batch_requests", "queued", "arena_used", "arena_high_water",
                 "rebalances")]


assert ctypes.sizeof(aesgpu_msg) == 48
assert ctypes.sizeof(aesgpu_done) == 56 and ctypes.sizeof(aesgpu_request) == 40


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_1201_0398_amd/build.py` "
            f"(hipcc, gfx950).  There is no fallback path.")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, ci = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    u8p = ctypes.POINTER(ctypes.c_uint8)
    kp = ctypes.POINTER(aesgpu_key)
    sig = {
        "aesgpu_create": ([ctypes.POINTER(vp), ci], ci),
        "aesgpu_destroy": ([vp], None),
        "aesgpu_expand_key": ([u8p, sz, kp], ci),
        "aesgpu_ecb_encrypt": ([vp, kp, vp, vp, sz, vp], ci),
        "aesgpu_ecb_decrypt": ([vp, kp, vp, vp, sz, vp], ci),
        "aesgpu_ctr_xcrypt": ([vp, kp, u8p, ctypes.c_uint32, vp, vp, sz, vp], ci),
        "aesgpu_ctr_le128_xcrypt": ([vp, kp, u8p, ctypes.c_uint64, vp, vp, sz, vp], ci),
        "aesgpu_cbc_decrypt": ([vp, kp, u8p, vp, vp, sz, vp], ci),
        "aesgpu_batch_plan": ([vp, ctypes.POINTER(aesgpu_msg), sz,
                               ctypes.POINTER(aesgpu_batch_config), ctypes.POINTER(vp)], ci),
        "aesgpu_batch_run": ([vp, vp, sz, vp, sz, vp, sz, vp], ci),
        "aesgpu_batch_run_noalloc": ([vp, ctypes.POINTER(aesgpu_msg), sz,
                                      ctypes.POINTER(aesgpu_batch_config), vp, sz, vp, sz, vp,
                                      sz, vp], ci),
        "aesgpu_batch_info": ([vp, ctypes.POINTER(aesgpu_batch_stats)], ci),
        "aesgpu_batch_free": ([vp], None),
        "aesgpu_arena_create": ([ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(vp)], ci),
        "aesgpu_arena_alloc": ([vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)], ci),
        "aesgpu_arena_release": ([vp, ctypes.c_uint64, ctypes.c_uint64], ci),
        "aesgpu_arena_query": ([vp] + [ctypes.POINTER(ctypes.c_uint64)] * 3, ci),
        "aesgpu_arena_destroy": ([vp], None),
        "aesgpu_server_create": ([vp, u8p, ctypes.POINTER(ctypes.c_uint16), sz,
                                  ctypes.POINTER(aesgpu_server_config), ctypes.POINTER(vp)], ci),
        "aesgpu_server_now": ([vp], ctypes.c_double),
        "aesgpu_server_submit": ([vp, ctypes.c_uint64, ci, ctypes.c_uint32, vp, sz,
                                  ctypes.c_double], ci),
        "aesgpu_server_poll": ([vp, ctypes.POINTER(aesgpu_done), sz, ctypes.POINTER(sz)], ci),
        "aesgpu_server_release": ([vp, vp, sz], ci),
        "aesgpu_server_get_stats": ([vp, ctypes.POINTER(aesgpu_server_stats)], ci),
        "aesgpu_server_replay": ([vp, ctypes.POINTER(aesgpu_request), sz, ctypes.c_double,
                                  ctypes.POINTER(aesgpu_done)], ci),
        "aesgpu_server_destroy": ([vp], None),
        "aesgpu_host_alloc": ([sz, ctypes.POINTER(vp)], ci),
        "aesgpu_host_free": ([vp], ci),
        "aesgpu_pipeline_create": ([vp, sz, ci, ctypes.c_uint32, ctypes.POINTER(vp)], ci),
        "aesgpu_pipeline_run": ([vp, kp, ctypes.POINTER(aesgpu_host_op), vp, vp, sz], ci),
        "aesgpu_pipeline_destroy": ([vp], None),
        "aesgpu_strerror": ([ci], ctypes.c_char_p),
        "aesgpu_ctx_num_cus": ([vp], ci),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


_lib: ctypes.CDLL | None = None
_lib = _load()


def lib() -> ctypes.CDLL:
    return _lib


def _check(status: int, what: str) -> int:
    if status != AESGPU_OK:
        raise AesgpuError(status, what)
    return status


def _ptr(x, need: int = 0) -> int | None:
    """Device address of a tensor (or an integer address as given).  A tensor
    must hold at least ``need`` bytes: the library takes plain pointers and
    cannot see a buffer's end, so a short tensor is refused here."""
    if x is None:
        return None
    if type(x) is torch.Tensor or isinstance(x, torch.Tensor):
        if not x.is_cuda:
            raise ValueError("buffer must be a device tensor")
        if not x.is_contiguous():
            raise ValueError("buffer must be contiguous")
        if x.nbytes < need:
            raise ValueError(f"buffer holds {x.nbytes} bytes, the call needs {need}")
        return x.data_ptr()
    if isinstance(x, int):
        return x
    raise TypeError(f"expected a device tensor or an address, got {type(x)}")


def _nbytes(x) -> int:
    return x.nbytes


# The current stream of the current device as a raw handle.  torch's own
# entry points for it are far cheaper per call than building a Stream object
# (torch.cuda.current_stream(), about 3 us), which bounds small calls.
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)
_cur_device = getattr(torch._C, "_cuda_getDevice", None)


def _stream(stream) -> int | None:
    if stream is None:
        if _raw_stream is not None and _cur_device is not None:
            return _raw_stream(_cur_device())
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _u8buf(b, n: int):
    raw = bytes(b)
    if len(raw) != n:
        raise ValueError(f"expected {n} bytes, got {len(raw)}")
    return (ctypes.c_uint8 * n).from_buffer_copy(raw)


# ---- context and keys --------------------------------------------------------

def aesgpu_create(device: int | None = None) -> ctypes.c_void_p:
    if device is None:
        device = torch.cuda.current_device()
    h = ctypes.c_void_p()
    _check(_lib.aesgpu_create(ctypes.byref(h), int(device)), "aesgpu_create")
    return h


def aesgpu_destroy(ctx) -> None:
    _lib.aesgpu_destroy(ctx)


def aesgpu_expand_key(key) -> aesgpu_key:
    raw = bytes(key)
    k = aesgpu_key()
    buf = (ctypes.c_uint8 * max(len(raw), 1)).from_buffer_copy(raw or b"\0")
    _check(_lib.aesgpu_expand_key(buf, len(raw), ctypes.byref(k)), "aesgpu_expand_key")
    return k


def aesgpu_strerror(status: int) -> str:
    return _lib.aesgpu_strerror(status).decode()


def aesgpu_ctx_num_cus(ctx) -> int:
    return int(_lib.aesgpu_ctx_num_cus(ctx))


# ---- single-buffer calls -------------------------------------------------------
# Each takes the same arguments as its C function; n_blocks / n_bytes default to
# the size of d_in.  ``check=False`` returns the status instead of raising.

def aesgpu_ecb_encrypt(ctx, key: aesgpu_key, d_in, d_out, n_blocks: int | None = None,
                       stream=None, check: bool = True) -> int:
    if n_blocks is None:
        n_blocks = _nbytes(d_in) // 16
    st = _lib.aesgpu_ecb_encrypt(ctx, ctypes.byref(key), _ptr(d_in, 16 * n_blocks),
                                 _ptr(d_out, 16 * n_blocks), n_blocks,
                                 _stream(stream))
    return _check(st, "aesgpu_ecb_encrypt") if check else st


def aesgpu_ecb_decrypt(ctx, key: aesgpu_key, d_in, d_out, n_blocks: int | None = None,
                       stream=None, check: bool = True) -> int:
    if n_blocks is None:
        n_blocks = _nbytes(d_in) // 16
    st = _lib.aesgpu_ecb_decrypt(ctx, ctypes.byref(key), _ptr(d_in, 16 * n_blocks),
                                 _ptr(d_out, 16 * n_blocks), n_blocks,
                                 _stream(stream))
    return _check(st, "aesgpu_ecb_decrypt") if check else st


def aesgpu_ctr_xcrypt(ctx, key: aesgpu_key, nonce, ctr0: int, d_in, d_out,
                      n_bytes: int | None = None, stream=None, check: bool = True) -> int:
    if n_bytes is None:
        n_bytes = _nbytes(d_in)
    st = _lib.aesgpu_ctr_xcrypt(ctx, ctypes.byref(key), _u8buf(nonce, 12), ctr0,
                                _ptr(d_in, n_bytes), _ptr(d_out, n_bytes), n_bytes,
                                _stream(stream))
    return _check(st, "aesgpu_ctr_xcrypt") if check else st


def aesgpu_ctr_le128_xcrypt(ctx, key: aesgpu_key, iv, index0: int, d_in, d_out,
                            n_bytes: int | None = None, stream=None, check: bool = True) -> int:
    if n_bytes is None:
        n_bytes = _nbytes(d_in)
    st = _lib.aesgpu_ctr_le128_xcrypt(ctx, ctypes.byref(key), _u8buf(iv, 16), index0,
                                      _ptr(d_in, n_bytes), _ptr(d_out, n_bytes), n_bytes,
                                      _stream(stream))
    return _check(st, "aesgpu_ctr_le128_xcrypt") if check else st


def aesgpu_cbc_decrypt(ctx, key: aesgpu_key, iv, d_in, d_out, n_blocks: int | None = None,
                       stream=None, check: bool = True) -> int:
    if n_blocks is None:
        n_blocks = _nbytes(d_in) // 16
    st = _lib.aesgpu_cbc_decrypt(ctx, ctypes.byref(key), _u8buf(iv, 16),
                                 _ptr(d_in, 16 * n_blocks), _ptr(d_out, 16 * n_blocks),
                                 n_blocks, _stream(stream))
    return _check(st, "aesgpu_cbc_decrypt") if check else st


# ---- batched messages ------------------------------------------------------------

def make_msgs(in_off, out_off, n_bytes, key_slot, key_bits, mode, dir, nonce=None, ctr0=None,
              iv=None):
    """Array of ``aesgpu_msg`` from per-message sequences (numpy or lists);
    ``nonce`` is an (m, 12) uint8 array.  ``iv`` (an (m, 16) uint8 array, for
    CBC messages) fills the 16 bytes from ``nonce`` on, i.e. nonce and ctr0;
    it is applied to the rows whose mode is CBC."""
    import numpy as np
    m = len(n_bytes)
    arr = (aesgpu_msg * m)()
    raw = np.frombuffer(arr, dtype=np.uint8).reshape(m, 48)
    view = raw.view(np.dtype([("in_off", "<u8"), ("out_off", "<u8"), ("n_bytes", "<u8"),
                              ("key_slot", "<u4"), ("key_bits", "<u2"), ("mode", "u1"),
                              ("dir", "u1"), ("nonce", "u1", (12,)), ("ctr0", "<u4")])).reshape(m)
    view["in_off"] = in_off
    view["out_off"] = out_off
    view["n_bytes"] = n_bytes
    view["key_slot"] = key_slot
    view["key_bits"] = key_bits
    view["mode"] = mode
    view["dir"] = dir
    if nonce is not None:
        view["nonce"] = nonce
    view["ctr0"] = 1 if ctr0 is None else ctr0
    if iv is not None:
        cbc = np.asarray(mode) == AESGPU_MODE_CBC
        ivs = np.asarray(iv, dtype=np.uint8).reshape(m, 16)
        raw[cbc, 32:48] = ivs[cbc]
    return arr


def aesgpu_batch_plan(ctx, msgs, blocks_per_lane: int = 0, tile_blocks: int = 0,
                      flags: int = 0, check: bool = True):
    """Returns a plan handle (or the status when ``check`` is False and it fails)."""
    cfg = aesgpu_batch_config(blocks_per_lane, tile_blocks, flags)
    h = ctypes.c_void_p()
    st = _lib.aesgpu_batch_plan(ctx, msgs, len(msgs), ctypes.byref(cfg), ctypes.byref(h))
    if check:
        _check(st, "aesgpu_batch_plan")
        return h
    return h if st == AESGPU_OK else st


def aesgpu_batch_run(plan, d_keys, n_key_slots: int, d_in, d_out, in_bytes: int | None = None,
                     out_bytes: int | None = None, stream=None, check: bool = True) -> int:
    if in_bytes is None:
        in_bytes = _nbytes(d_in)
    if out_bytes is None:
        out_bytes = _nbytes(d_out)
    st = _lib.aesgpu_batch_run(plan, _ptr(d_keys, 32 * n_key_slots), n_key_slots,
                               _ptr(d_in, in_bytes), in_bytes, _ptr(d_out, out_bytes),
                               out_bytes, _stream(stream))
    return _check(st, "aesgpu_batch_run") if check else st


def aesgpu_batch_run_noalloc(ctx, msgs, d_keys, n_key_slots: int, d_in, d_out,
                             in_bytes: int | None = None, out_bytes: int | None = None,
                             blocks_per_lane: int = 0, tile_blocks: int = 0, stream=None,
                             check: bool = True) -> int:
    """Plans and runs one batch with no device allocation (the library's
    fixed per-GPU scratch holds the descriptors)."""
    if in_bytes is None:
        in_bytes = _nbytes(d_in)
    if out_bytes is None:
        out_bytes = _nbytes(d_out)
    cfg = aesgpu_batch_config(blocks_per_lane, tile_blocks, 0)
    st = _lib.aesgpu_batch_run_noalloc(ctx, msgs, len(msgs), ctypes.byref(cfg),
                                       _ptr(d_keys, 32 * n_key_slots), n_key_slots,
                                       _ptr(d_in, in_bytes), in_bytes, _ptr(d_out, out_bytes),
                                       out_bytes, _stream(stream))
    return _check(st, "aesgpu_batch_run_noalloc") if check else st


def aesgpu_batch_info(plan) -> aesgpu_batch_stats:
    st = aesgpu_batch_stats()
    _check(_lib.aesgpu_batch_info(plan, ctypes.byref(st)), "aesgpu_batch_info")
    return st


def aesgpu_batch_free(plan) -> None:
    _lib.aesgpu_batch_free(plan)


# ---- range allocator ---------------------------------------------------------------

def aesgpu_arena_create(capacity: int, granule: int = 256):
    h = ctypes.c_void_p()
    _check(_lib.aesgpu_arena_create(capacity, granule, ctypes.byref(h)), "aesgpu_arena_create")
    return h


def aesgpu_arena_alloc(arena, n_bytes: int):
    """Offset of the new range, or None when nothing fits right now (EAGAIN)."""
    off = ctypes.c_uint64()
    st = _lib.aesgpu_arena_alloc(arena, n_bytes, ctypes.byref(off))
    if st == AESGPU_EAGAIN:
        return None
    _check(st, "aesgpu_arena_alloc")
    return off.value


def aesgpu_arena_release(arena, offset: int, n_bytes: int, check: bool = True) -> int:
    st = _lib.aesgpu_arena_release(arena, offset, n_bytes)
    return _check(st, "aesgpu_arena_release") if check else st


def aesgpu_arena_query(arena) -> tuple[int, int, int]:
    """(used, largest free range, high-water mark) in bytes."""
    u, f, h = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(_lib.aesgpu_arena_query(arena, ctypes.byref(u), ctypes.byref(f), ctypes.byref(h)),
           "aesgpu_arena_query")
    return u.value, f.value, h.value


def aesgpu_arena_destroy(arena) -> None:
    _lib.aesgpu_arena_destroy(arena)


# ---- serving ------------------------------------------------------------------------

def aesgpu_server_create(ctx, keys, key_bits, arena_bytes: int, n_streams: int = 0,
                         blocks_per_lane: int = 0, tile_blocks: int = 0,
                         max_batch_requests: int = 0, max_batch_bytes: int = 0,
                         max_queued: int = 0, direct_requests: int = 0, flags: int = 0):
    """keys: (n, 32) uint8 host array (key bytes first); key_bits: n sizes."""
    import numpy as np
    k = np.ascontiguousarray(keys, dtype=np.uint8).reshape(-1, 32)
    bits = np.ascontiguousarray(key_bits, dtype=np.uint16).reshape(-1)
    assert bits.size == k.shape[0]
    cfg = aesgpu_server_config(arena_bytes, n_streams, blocks_per_lane, tile_blocks,
                               max_batch_requests, max_batch_bytes, max_queued,
                               direct_requests, flags)
    h = ctypes.c_void_p()
    _check(_lib.aesgpu_server_create(ctx, k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                     bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                     bits.size, ctypes.byref(cfg), ctypes.byref(h)),
           "aesgpu_server_create")
    return h


def aesgpu_server_now(server) -> float:
    return float(_lib.aesgpu_server_now(server))


def aesgpu_server_submit(server, req_id: int, dir: int, key_id: int, d_in, n_bytes=None,
                         t_arrival: float | None = None, check: bool = True) -> int:
    if n_bytes is None:
        n_bytes = _nbytes(d_in)
    if t_arrival is None:
        t_arrival = aesgpu_server_now(server)
    st = _lib.aesgpu_server_submit(server, req_id, dir, key_id, _ptr(d_in, n_bytes), n_bytes,
                                   t_arrival)
    return _check(st, "aesgpu_server_submit") if check else st


def aesgpu_server_poll(server, cap: int = 1024) -> list:
    buf = (aesgpu_done * cap)()
    n = ctypes.c_size_t()
    _check(_lib.aesgpu_server_poll(server, buf, cap, ctypes.byref(n)), "aesgpu_server_poll")
    return [buf[i] for i in range(n.value)]


def aesgpu_server_release(server, d_out, n_bytes: int) -> int:
    return _check(_lib.aesgpu_server_release(server, d_out, n_bytes), "aesgpu_server_release")


def aesgpu_server_get_stats(server) -> aesgpu_server_stats:
    st = aesgpu_server_stats()
    _check(_lib.aesgpu_server_get_stats(server, ctypes.byref(st)), "aesgpu_server_get_stats")
    return st


def aesgpu_server_replay(server, reqs, t_start: float):
    """reqs: ctypes array of aesgpu_request; returns a ctypes array of
    aesgpu_done indexed by req_id."""
    n = len(reqs)
    done = (aesgpu_done * n)()
    _check(_lib.aesgpu_server_replay(server, reqs, n, t_start, done), "aesgpu_server_replay")
    return done


def make_requests(t_arrival, d_in, n_bytes, key_id, dir):
    """Array of ``aesgpu_request`` (req_id = position) from per-request
    sequences; ``d_in`` holds device addresses."""
    import numpy as np
    n = len(n_bytes)
    arr = (aesgpu_request * n)()
    view = np.frombuffer(arr, dtype=np.dtype(
        [("req_id", "<u8"), ("t_arrival", "<f8"), ("d_in", "<u8"), ("n_bytes", "<u8"),
         ("key_id", "<u4"), ("dir", "<u4")]), count=n)
    view["req_id"] = np.arange(n)
    view["t_arrival"] = t_arrival
    view["d_in"] = d_in
    view["n_bytes"] = n_bytes
    view["key_id"] = key_id
    view["dir"] = dir
    return arr


def aesgpu_server_destroy(server) -> None:
    _lib.aesgpu_server_destroy(server)


# ---- host-staged pipeline ----------------------------------------------------

def aesgpu_host_alloc(n_bytes: int):
    """Pinned host memory; returns (address, numpy uint8 view of n_bytes)."""
    import numpy as np
    p = ctypes.c_void_p()
    _check(_lib.aesgpu_host_alloc(n_bytes, ctypes.byref(p)), "aesgpu_host_alloc")
    view = np.ctypeslib.as_array((ctypes.c_uint8 * n_bytes).from_address(p.value))
    return p.value, view


def aesgpu_host_free(addr: int, check: bool = True) -> int:
    st = _lib.aesgpu_host_free(addr)
    return _check(st, "aesgpu_host_free") if check else st


def _host_ptr(x, need: int = 0) -> int | None:
    """Host address of a contiguous numpy array of at least ``need`` bytes
    (or an integer address)."""
    if x is None or isinstance(x, int):
        return x
    import numpy as np
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("host buffer must be contiguous")
        if x.nbytes < need:
            raise ValueError(f"host buffer holds {x.nbytes} bytes, the call needs {need}")
        return x.ctypes.data
    raise TypeError(f"expected a numpy array or an address, got {type(x)}")


def make_host_op(op: int, ctr0: int = 0, nonce=None, iv=None) -> aesgpu_host_op:
    o = aesgpu_host_op()
    o.op = op
    o.ctr0 = ctr0
    if nonce is not None:
        o.nonce[:] = bytes(nonce)
    if iv is not None:
        o.iv[:] = bytes(iv)
    return o


AESGPU_PIPELINE_COPY = 1


def aesgpu_pipeline_create(ctx, chunk_bytes: int = 0, n_slots: int = 0, flags: int = 0):
    out = ctypes.c_void_p()
    _check(_lib.aesgpu_pipeline_create(ctx, chunk_bytes, n_slots, flags, ctypes.byref(out)),
           "aesgpu_pipeline_create")
    return out


def aesgpu_pipeline_run(pl, key: aesgpu_key, op: aesgpu_host_op, h_in, h_out,
                        n_bytes: int | None = None, check: bool = True) -> int:
    if n_bytes is None:
        n_bytes = h_in.nbytes
    st = _lib.aesgpu_pipeline_run(pl, ctypes.byref(key), ctypes.byref(op),
                                  _host_ptr(h_in, n_bytes), _host_ptr(h_out, n_bytes), n_bytes)
    return _check(st, "aesgpu_pipeline_run") if check else st


def aesgpu_pipeline_destroy(pl) -> None:
    _lib.aesgpu_pipeline_destroy(pl)
