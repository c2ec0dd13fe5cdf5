"""Writes ``full_size_digests.json``: SHA-256 digests of the CPU oracle's
outputs over the whole full-size workloads, so that a GPU test can compare
every output byte with the oracle without re-running the (slow, literal)
oracle on the GPU machine.

Workloads (``paper_1201_0398_amd.workloads``):

* 1 GiB, seed 1: ECB encryption and ECB decryption of the random buffer with
  each of the three keys, and AES-128 CTR (nonce || BE32 counter from 1);
* the same buffer decrypted in CBC mode with the AES-128 and AES-256 keys, IV
  = the workload's nonce followed by its ctr0 as 4 big-endian bytes;
* the same buffer through the paper's LE-128 counter mode with the AES-192 key:
  IV = 2^32 - 2^25 as 4 little-endian bytes (so counter word 0 wraps in the
  middle of the buffer) followed by the nonce, block index from 0;
* 4 GiB, seed 2: AES-256 CTR from counter 1, in 256 MiB chunks (the counter
  advances by 2^24 per chunk);
* 65,536 messages, seed 3: the packed output buffer of the encryption run
  and of the decryption run (every message decrypted: ECB messages through
  the inverse cipher, CTR messages through the same keystream);
* 65,536 CBC messages, seed 6 (``workloads.cbc_batch``): the packed output of
  CBC encryption of every message, and of CBC decryption of the same input
  bytes taken as ciphertext.

Calls only the oracle and the seeded input generators.  Takes about half an
hour on 8 cores.  Run from the repository root:
``python tests/golden/make_full_digests.py [--only NAME ...]``.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1201_0398_amd import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_digests.json")
CHUNK = 1 << 28   # 256 MiB = 2^24 blocks


def sha(a) -> str:
    return hashlib.sha256(memoryview(np.ascontiguousarray(a))).hexdigest()


def log(msg: str) -> None:
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def gib1(out: dict) -> None:
    w = workloads.single_1gib(seed=1)
    out["gib1_input_sha256"] = sha(w.data)
    for bits in (128, 192, 256):
        key = w.keys[bits]
        log(f"1 GiB ECB-{bits} encrypt")
        out[f"gib1_ecb{bits}_encrypt_sha256"] = sha(oracle.ecb_encrypt(key, w.data))
        log(f"1 GiB ECB-{bits} decrypt")
        out[f"gib1_ecb{bits}_decrypt_sha256"] = sha(oracle.ecb_decrypt(key, w.data))
    log("1 GiB CTR-128")
    out["gib1_ctr128_sha256"] = sha(oracle.ctr(w.keys[128], w.nonce, w.ctr0, w.data))


def cbc_iv(w) -> np.ndarray:
    """The CBC IV of the 1 GiB workload: its 12-byte nonce, then ctr0 as 4
    big-endian bytes (a fixed derivation from the seeded inputs)."""
    return np.concatenate([np.asarray(w.nonce, dtype=np.uint8),
                           np.frombuffer(int(w.ctr0).to_bytes(4, "big"), dtype=np.uint8)])


def gib1_cbc(out: dict) -> None:
    w = workloads.single_1gib(seed=1)
    for bits in (128, 256):
        log(f"1 GiB CBC-{bits} decrypt")
        out[f"gib1_cbc{bits}_decrypt_sha256"] = sha(oracle.cbc_decrypt(w.keys[bits], cbc_iv(w),
                                                                       w.data))


def le128_iv(w) -> np.ndarray:
    """The LE-128 CTR IV of the 1 GiB workload: word 0 = 2^32 - 2^25 (it
    wraps after 2^25 of the buffer's 2^26 blocks), words 1..3 = the nonce."""
    return np.concatenate([np.frombuffer((2**32 - 2**25).to_bytes(4, "little"), dtype=np.uint8),
                           np.asarray(w.nonce, dtype=np.uint8)])


def gib1_le128(out: dict) -> None:
    w = workloads.single_1gib(seed=1)
    log("1 GiB LE-128 CTR-192")
    out["gib1_ctrle128_192_sha256"] = sha(oracle.ctr_le128(w.keys[192], le128_iv(w), 0, w.data))


def gib4(out: dict) -> None:
    w = workloads.ctr_4gib(seed=2)
    out["gib4_input_sha256"] = sha(w.data)
    h = hashlib.sha256()
    for i, o in enumerate(range(0, w.data.size, CHUNK)):
        log(f"4 GiB CTR-256 chunk {i}")
        h.update(memoryview(oracle.ctr(w.keys[256], w.nonce, w.ctr0 + i * (CHUNK // 16),
                                       w.data[o:o + CHUNK])))
    out["gib4_ctr256_sha256"] = h.hexdigest()


def batched(out: dict) -> None:
    w = workloads.batched(seed=3)
    m = w.lengths.size
    out["batched_input_sha256"] = sha(w.data)
    out["batched_total_bytes"] = int(w.total_bytes)
    enc = np.empty_like(w.data)
    dec = np.empty_like(w.data)
    t0 = time.time()
    for j in range(m):
        o, L = int(w.offsets[j]), int(w.lengths[j])
        key = w.keys[j, : int(w.key_bits[j]) // 8]
        src = w.data[o:o + L]
        if w.modes[j]:
            enc[o:o + L] = oracle.ctr(key, w.nonces[j], int(w.ctr0[j]), src)
            dec[o:o + L] = enc[o:o + L]
        else:
            enc[o:o + L] = oracle.ecb_encrypt(key, src)
            dec[o:o + L] = oracle.ecb_decrypt(key, src)
        if j % 8192 == 8191:
            log(f"batched: {j + 1} of {m} messages ({time.time() - t0:.0f} s)")
    out["batched_encrypt_sha256"] = sha(enc)
    out["batched_decrypt_sha256"] = sha(dec)


def cbc_batch(out: dict) -> None:
    w = workloads.cbc_batch(seed=6)
    m = w.lengths.size
    out["cbc_batch_input_sha256"] = sha(w.data)
    enc = np.empty_like(w.data)
    dec = np.empty_like(w.data)
    t0 = time.time()
    for j in range(m):
        o, L = int(w.offsets[j]), int(w.lengths[j])
        key = w.keys[j, : int(w.key_bits[j]) // 8]
        enc[o:o + L] = oracle.cbc_encrypt(key, w.ivs[j], w.data[o:o + L])
        dec[o:o + L] = oracle.cbc_decrypt(key, w.ivs[j], w.data[o:o + L])
        if j % 16384 == 16383:
            log(f"CBC batch: {j + 1} of {m} messages ({time.time() - t0:.0f} s)")
    out["cbc_batch_encrypt_sha256"] = sha(enc)
    out["cbc_batch_decrypt_sha256"] = sha(dec)


PARTS = {"gib1": gib1, "gib1_cbc": gib1_cbc, "gib1_le128": gib1_le128, "gib4": gib4,
         "batched": batched, "cbc_batch": cbc_batch}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", choices=sorted(PARTS), default=sorted(PARTS))
    args = ap.parse_args()
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    out["recipe"] = ("workloads.single_1gib(seed=1), workloads.ctr_4gib(seed=2), "
                     "workloads.batched(seed=3), workloads.cbc_batch(seed=6); "
                     "digests of whole oracle outputs")
    for name in args.only:
        PARTS[name](out)
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")
        log(f"{name} written")


if __name__ == "__main__":
    main()
