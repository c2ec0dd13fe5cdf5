"""Stored oracle digests (written by ``golden/make_golden.py`` from the oracle
alone) still match: guards the oracle and the input recipe against drift."""
import hashlib
import json
import os

import oracle
from paper_1201_0398_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")


def _sha(a):
    return hashlib.sha256(bytes(a)).hexdigest()


def test_oracle_digests_small_workload():
    with open(GOLDEN) as f:
        g = json.load(f)
    w = workloads.single_small(seed=0)
    assert _sha(w.data) == g["input_sha256"]
    key = w.keys[128]
    assert _sha(oracle.ecb_encrypt(key, w.data)) == g["ecb128_encrypt_sha256"]
    assert _sha(oracle.ecb_decrypt(key, w.data)) == g["ecb128_decrypt_of_input_sha256"]
    assert _sha(oracle.ctr(key, w.nonce, w.ctr0, w.data)) == g["ctr128_sha256"]
    assert _sha(w.iv) == g["iv_sha256"]
    assert _sha(oracle.ctr_le128(key, w.iv, 0, w.data)) == g["ctr_le128_index0_0_sha256"]
    assert _sha(oracle.cbc_encrypt(key, w.iv, w.data)) == g["cbc128_encrypt_sha256"]
    assert _sha(oracle.cbc_decrypt(key, w.iv, w.data)) == g["cbc128_decrypt_of_input_sha256"]


def test_full_size_input_recipe():
    """The 1 GiB workload's input still hashes to the digest the full-size
    oracle digests were computed on (golden/full_size_digests.json)."""
    with open(os.path.join(os.path.dirname(GOLDEN), "full_size_digests.json")) as f:
        g = json.load(f)
    w = workloads.single_1gib(seed=1)
    assert hashlib.sha256(memoryview(w.data)).hexdigest() == g["gib1_input_sha256"]
