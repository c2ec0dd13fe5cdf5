"""Host-side checks of the C ABI (no GPU needed): exported symbols, key
expansion against the oracle, and argument errors detected before any HIP
call."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")
LIB = os.path.join(ROOT, "paper_1201_0398_amd", "libaesgpu.so")


def _declared_functions():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if fn.endswith(".h"):
            text = open(os.path.join(HEADER_DIR, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(aesgpu_\w+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def A():
    if not os.path.exists(LIB):
        from paper_1201_0398_amd import build
        build.build()
    from paper_1201_0398_amd import aesgpu
    return aesgpu


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["aesgpu_create", "aesgpu_destroy", "aesgpu_expand_key", "aesgpu_ecb_encrypt",
                     "aesgpu_ecb_decrypt", "aesgpu_ctr_xcrypt", "aesgpu_strerror"]:
        assert required in names


def test_library_exports_every_declared_symbol(A):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (aesgpu_\w+)", out))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    lib = A.lib()
    for n in _declared_functions():
        assert hasattr(lib, n)


@pytest.mark.parametrize("kb", [16, 24, 32])
def test_expand_key_matches_oracle(A, kb):
    rng = np.random.default_rng(100 + kb)
    for _ in range(20):
        key = rng.integers(0, 256, kb, dtype=np.uint8)
        k = A.aesgpu_expand_key(bytes(key))
        nr = kb // 4 + 6
        assert k.key_bits == 8 * kb and k.nr == nr
        w = oracle.key_expansion(key)                 # (4*(nr+1), 4) bytes
        enc = np.array(k.enc[: 4 * (nr + 1)], dtype=np.uint32)
        want = w.astype(np.uint32) @ np.array([1, 1 << 8, 1 << 16, 1 << 24], dtype=np.uint32)
        assert np.array_equal(enc, want)
        # Decryption keys: round r = InvMixColumns(enc round nr - r), except ends.
        dec = np.array(k.dec[: 4 * (nr + 1)], dtype=np.uint32).view(np.uint8).reshape(nr + 1, 16)
        rounds = w.reshape(nr + 1, 16)
        for r in range(nr + 1):
            src = rounds[nr - r]
            want_r = src if r in (0, nr) else oracle.transform("inv_mix_columns", src)
            assert np.array_equal(dec[r], want_r), f"dec round {r}"


def test_expand_key_errors(A):
    for n in (0, 8, 15, 17, 31, 33):
        with pytest.raises(A.AesgpuError) as e:
            A.aesgpu_expand_key(bytes(n))
        assert e.value.status in (A.AESGPU_EKEYLEN, A.AESGPU_EINVAL)
    k = A.aesgpu_key()
    assert A.lib().aesgpu_expand_key(None, 16, ctypes.byref(k)) == A.AESGPU_EINVAL


def test_calls_reject_null_context_before_any_hip_call(A):
    k = A.aesgpu_expand_key(bytes(16))
    L = A.lib()
    kp = ctypes.byref(k)
    nonce = (ctypes.c_uint8 * 16)()
    assert L.aesgpu_ecb_encrypt(None, kp, 16, 16, 1, None) == A.AESGPU_EINVAL
    assert L.aesgpu_ecb_decrypt(None, kp, 16, 16, 1, None) == A.AESGPU_EINVAL
    assert L.aesgpu_ctr_xcrypt(None, kp, nonce, 1, 16, 16, 16, None) == A.AESGPU_EINVAL
    assert L.aesgpu_ctr_le128_xcrypt(None, kp, nonce, 0, 16, 16, 16, None) == A.AESGPU_EINVAL
    assert L.aesgpu_cbc_decrypt(None, kp, nonce, 16, 32, 1, None) == A.AESGPU_EINVAL
    out = ctypes.c_void_p()
    assert L.aesgpu_pipeline_create(None, 0, 0, 0, ctypes.byref(out)) == A.AESGPU_EINVAL
    assert out.value is None
    op = A.make_host_op(A.AESGPU_OP_ECB_ENCRYPT)
    assert L.aesgpu_pipeline_run(None, kp, ctypes.byref(op), 16, 32, 16) == A.AESGPU_EINVAL
    assert L.aesgpu_host_alloc(0, ctypes.byref(out)) == A.AESGPU_EINVAL
    assert L.aesgpu_host_free(4096) == A.AESGPU_EINVAL     # not from aesgpu_host_alloc
    assert L.aesgpu_host_free(None) == A.AESGPU_OK
    L.aesgpu_pipeline_destroy(None)


def test_strerror_names_every_code(A):
    for st in range(-7, 1):
        assert A.aesgpu_strerror(st) and A.aesgpu_strerror(st) != "unknown status"
    assert A.aesgpu_strerror(-99) == "unknown status"


STRUCTS = ["aesgpu_key", "aesgpu_msg", "aesgpu_batch_config", "aesgpu_batch_stats",
           "aesgpu_server_config", "aesgpu_done", "aesgpu_request", "aesgpu_host_op",
           "aesgpu_server_stats"]


def test_binding_structs_match_the_header(A, tmp_path):
    """Every ctypes mirror has the C struct's size and each field's offset,
    as a C compiler lays them out from include/aesgpu.h."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "aesgpu.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(A, name)
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", HEADER_DIR, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    c_layout = {}
    for line in out.splitlines():
        name, field, value = line.split()
        c_layout[(name, field)] = int(value)
    for name in STRUCTS:
        cls = getattr(A, name)
        assert ctypes.sizeof(cls) == c_layout[(name, "sizeof")], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == c_layout[(name, field)], f"{name}.{field}"
