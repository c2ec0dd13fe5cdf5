"""The library's host code under sanitizers, on the CPU (no GPU needed).

``native/host_checks.cpp`` drives the host-only logic: key expansion,
argument validation, the batch planner, the allocation-free batch call's
host staging, the server's range allocator and the pipeline's host copy
pool.  It is built twice with hipcc, the sanitizers applied to host code
only: with AddressSanitizer + UndefinedBehaviorSanitizer (every check), and
with ThreadSanitizer (the copy pool's worker threads, several pools at once,
and one range allocator shared by threads under a lock).  Each build must
report no error and every check must hold."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1201_0398_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
DRIVER = os.path.join(ROOT, "tests", "native", "host_checks.cpp")

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")

# Host-side sanitizer flags; each -fsanitize= applies to host code only.
SANITIZERS = {
    "asan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"],
    "tsan": ["-Xarch_host", "-fsanitize=thread"],
}


def build(kind: str, out_dir: str) -> str:
    flags = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SANITIZERS[kind]]
    units = [(os.path.join(CSRC, "aes_host.cpp"), []), (os.path.join(CSRC, "aes_server.cpp"), []),
             (os.path.join(CSRC, "aes_kernels.hip"), ["-x", "hip"]),
             (os.path.join(CSRC, "aes_batch.hip"), ["-x", "hip"]), (DRIVER, [])]
    procs, objs = [], []
    for src, lang in units:
        obj = os.path.join(out_dir, f"{kind}_{os.path.splitext(os.path.basename(src))[0]}.o")
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *flags, *lang, "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, f"compile failed:\n{out[-4000:]}"
    exe = os.path.join(out_dir, f"host_checks_{kind}")
    subprocess.run([HIPCC, "--offload-arch=gfx950", *SANITIZERS[kind], *objs, "-o", exe],
                   check=True, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    return exe


@pytest.mark.parametrize("kind", ["asan", "tsan"])
def test_host_code_under_sanitizer(kind, tmp_path):
    exe = build(kind, str(tmp_path))
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=24"
    env["TSAN_OPTIONS"] = "halt_on_error=1:exitcode=25"
    r = subprocess.run([exe, kind], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, env=env,
                       timeout=300)
    out = r.stdout.decode(errors="replace")
    print(out[-2000:], file=sys.stderr)
    assert r.returncode == 0, f"{kind} run failed ({r.returncode}):\n{out[-6000:]}"
    assert f"host checks ok ({kind})" in out
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out
    assert "WARNING: ThreadSanitizer" not in out
    shutil.rmtree(str(tmp_path), ignore_errors=True)
