"""Writes ``oracle_digests.json``: SHA-256 digests of oracle outputs on the
seeded 1 MiB workload (seed 0).  Calls only the CPU oracle and the seeded input
generators.  Run from the repository root: ``python tests/golden/make_golden.py``.
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1201_0398_amd import workloads  # noqa: E402


def sha(a) -> str:
    return hashlib.sha256(bytes(a)).hexdigest()


def main():
    w = workloads.single_small(seed=0)
    key = w.keys[128]
    enc = oracle.ecb_encrypt(key, w.data)
    out = {
        "workload": "1 MiB uniform random bytes, one AES-128 key, seed 0",
        "input_sha256": sha(w.data),
        "ecb128_encrypt_sha256": sha(enc),
        "ecb128_decrypt_of_input_sha256": sha(oracle.ecb_decrypt(key, w.data)),
        "ecb128_roundtrip_ok": bool((oracle.ecb_decrypt(key, enc) == w.data).all()),
        "ctr128_sha256": sha(oracle.ctr(key, w.nonce, w.ctr0, w.data)),
        "iv_sha256": sha(w.iv),
        "ctr_le128_index0_0_sha256": sha(oracle.ctr_le128(key, w.iv, 0, w.data)),
        "cbc128_encrypt_sha256": sha(oracle.cbc_encrypt(key, w.iv, w.data)),
        "cbc128_decrypt_of_input_sha256": sha(oracle.cbc_decrypt(key, w.iv, w.data)),
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_digests.json"),
              "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
