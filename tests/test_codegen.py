"""Properties of the generated gfx950 code that the kernels' speed rests on,
checked on the CPU from hipcc's own assembly of the library sources:

* the tile loop of every single-buffer kernel (each operation, key size and
  blocks-per-lane variant) is one basic block, with no branch inside: with any
  branch in that loop, uniform or not, the compiler's schedule keeps only about
  five LDS table reads in flight per wave instead of 12-17;
* the loop keeps many table reads in flight: the mean number of LDS reads
  outstanding at each wait for them is at least 7 / 10 / 10 at 1 / 2 / 4 blocks
  per lane;
* no kernel spills registers to scratch memory, apart from the variants listed
  in KNOWN_SPILLS (which the launch code avoids or which measured no faster
  without the spill);
* no single-buffer kernel sign-extends a scalar value: every index, count and
  address there is unsigned, and a 32-bit value sign-extended into the high
  word of a 64-bit buffer base address points outside the buffer.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

OPS = {"0": "ecb_enc", "1": "ecb_dec", "2": "ctr_be32", "3": "ctr_le128", "4": "cbc_dec"}
MIN_IN_FLIGHT = {1: 7.0, 2: 10.0, 4: 10.0}
# (op, Nr, blocks per lane) -> bytes of scratch per lane allowed.  AES-256 ECB
# and CTR at 4 blocks per lane reload a few words per tile (ECB measured no
# faster at 2); CBC decryption with AES-192/256 keys launches at 2 blocks per
# lane instead.
KNOWN_SPILLS = {("ecb_enc", 14, 4): 20, ("ecb_dec", 14, 4): 20, ("ctr_be32", 14, 4): 8,
                ("cbc_dec", 14, 4): 36}


def _asm(src: str, tmp_path) -> list:
    from paper_1201_0398_amd import build
    if not os.path.exists(build.HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = os.path.join(str(tmp_path), os.path.basename(src) + ".s")
    cmd = [build.HIPCC, *[f for f in build.HIP_FLAGS if f not in ("-fPIC", "-Wall")],
           "--cuda-device-only", "-S", "-I", build.INCLUDE, "-I", build.CSRC, "-x", "hip",
           os.path.join(build.CSRC, src), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    with open(out) as f:
        return f.read().split("\n")


def _kernels(lines: list):
    """(name, first line, end line) of every kernel symbol."""
    heads = [(i, l.split(":")[0]) for i, l in enumerate(lines) if re.match(r"^_Z\S+:", l)]
    for k, (i, name) in enumerate(heads):
        yield name, i, heads[k + 1][0] if k + 1 < len(heads) else len(lines)


def _largest_loop(lines: list, lo: int, hi: int):
    """The largest backward branch to a loop header (as the compiler's own
    annotation names it): the tile loop."""
    labels, best = {}, None
    for j in range(lo, hi):
        m = re.match(r"^(\.LBB\d+_\d+):", lines[j])
        if m and "Loop Header" in lines[j]:
            labels[m.group(1)] = j
        m = re.match(r"\s+s_(cbranch_\w+|branch)\s+(\.LBB\d+_\d+)", lines[j])
        if m and m.group(2) in labels and labels[m.group(2)] < j:
            s = labels[m.group(2)]
            if best is None or j - s > best[1] - best[0]:
                best = (s, j)
    return best


def _in_flight(body: list) -> float:
    """Mean number of LDS reads outstanding at each wait on the LDS counter."""
    n, at = 0, []
    for line in body:
        t = line.strip()
        if t.startswith("ds_read"):
            n += 1
        m = re.match(r"s_waitcnt.*lgkmcnt\((\d+)\)", t)
        if m:
            at.append(n)
            n = min(n, int(m.group(1)))
    return sum(at) / max(1, len(at))


def _scratch(lines: list, lo: int, hi: int) -> int:
    for j in range(lo, hi):
        m = re.search(r"; ScratchSize: (\d+)", lines[j])
        if m:
            return int(m.group(1))
    raise AssertionError("no ScratchSize note")


def test_single_buffer_tile_loops(tmp_path):
    lines = _asm("aes_kernels.hip", tmp_path)
    seen = 0
    for name, lo, hi in _kernels(lines):
        m = re.search(r"aes_kernelILNS_2OpE(\d)ELi(\d+)ELi(\d)ELb(\d)E", name)
        if not m:
            continue
        op, nr, bpl = OPS[m.group(1)], int(m.group(2)), int(m.group(3))
        if m.group(4) == "0":
            op += " (one share per wave)"
        seen += 1
        loop = _largest_loop(lines, lo, hi)
        assert loop is not None, f"{op} Nr={nr} {bpl}/lane: no tile loop"
        body = lines[loop[0] + 1:loop[1]]
        assert not any(re.match(r"^\.LBB\d+_\d+:", l) for l in body), \
            f"{op} Nr={nr} {bpl}/lane: the tile loop has more than one basic block"
        assert not any(re.match(r"\s+s_(cbranch_\w+|branch)\s", l) for l in body), \
            f"{op} Nr={nr} {bpl}/lane: a branch inside the tile loop"
        got = _in_flight(body)
        assert got >= MIN_IN_FLIGHT[bpl], \
            f"{op} Nr={nr} {bpl}/lane: {got:.1f} table reads in flight at a wait"
        assert _scratch(lines, lo, hi) <= KNOWN_SPILLS.get((op.split()[0], nr, bpl), 0), \
            f"{op} Nr={nr} {bpl}/lane spills to scratch"
        signed = [l.strip() for l in lines[lo:hi] if re.match(r"\s+s_(bfe_i64|bfe_i32|ashr_i32|ashr_i64|sext)", l)]
        assert not signed, f"{op} Nr={nr} {bpl}/lane sign-extends: {signed[:3]}"
    # every operation, key size and blocks per lane with shares claimed, and
    # at one block per lane also with one share per wave
    assert seen == 5 * 3 * 3 + 5 * 3, f"expected 60 single-buffer kernels, found {seen}"


def test_batched_kernels_do_not_spill(tmp_path):
    lines = _asm("aes_batch.hip", tmp_path)
    seen = 0
    for name, lo, hi in _kernels(lines):
        if "batch_kernel" in name or "resident_kernel" in name or "cbc_encrypt_kernel" in name:
            seen += 1
            assert _scratch(lines, lo, hi) == 0, f"{name} spills to scratch"
    assert seen >= 8
