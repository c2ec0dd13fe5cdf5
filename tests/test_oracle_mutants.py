"""Each plausible mistake planted in a copy of the oracle fails some pin.

The copies are built on the CPU from edited text of ``oracle/aes_oracle.c``; the
real oracle is never modified.  This shows that the pins in ``oracle_pins``
would catch a dropped term, a wrong constant, a wrong index or a transposed
operand anywhere in the oracle.
"""
import functools

import pytest

import oracle
import openssl_ref
import oracle_pins as P

# (name, text in aes_oracle.c, replacement)
MUTANTS = [
    ("modulus", "shifted ^= 0x1B;", "shifted ^= 0x1D;"),
    ("inverse_exponent", "unsigned e = 254;", "unsigned e = 253;"),
    ("affine_constant", "(0x63 >> i)", "(0x43 >> i)"),
    ("affine_rotation", "(b >> ((i + 4) & 7))", "(b >> ((i + 3) & 7))"),
    ("shift_rows_direction", "s[r][c] = t[r][(c + r) % 4];", "s[r][c] = t[r][(c + 4 - r) % 4];"),
    ("inv_shift_rows_direction", "s[r][(c + r) % 4] = t[r][c];", "s[r][c] = t[r][c];"),
    ("mix_row_transposed", "{0x02, 0x03, 0x01, 0x01}", "{0x03, 0x02, 0x01, 0x01}"),
    ("inv_mix_row", "{0x0E, 0x0B, 0x0D, 0x09}", "{0x0E, 0x09, 0x0D, 0x0B}"),
    ("circulant_transposed", "m[(k - r + 4) % 4]", "m[(r - k + 4) % 4]"),
    ("rotword", "{temp[1], temp[2], temp[3], temp[0]}", "{temp[3], temp[0], temp[1], temp[2]}"),
    ("rcon_index", "rcon_byte(i / nk)", "rcon_byte(i / nk + 1)"),
    ("aes256_subword_dropped", "nk > 6 && i % nk == 4", "nk > 8 && i % nk == 4"),
    ("ark_transposed", "s[r][c] ^= w[4 * round + c][r];", "s[r][c] ^= w[4 * round + r][c];"),
    ("final_round_no_shift",
     "    sub_bytes(s);\n    shift_rows(s);\n    add_round_key(s, w, nr);",
     "    sub_bytes(s);\n    add_round_key(s, w, nr);"),
    ("inv_cipher_order",
     "        add_round_key(s, w, round);\n        inv_mix_columns(s);",
     "        inv_mix_columns(s);\n        add_round_key(s, w, round);"),
    ("ttable_index", "TT.te[1][byte_of(I[(c + 1) % 4], 1)]", "TT.te[1][byte_of(I[(c + 3) % 4], 1)]"),
    ("td_key_no_invmix", "            inv_mix_columns(s);\n        for (int c = 0; c < 4; c++) {\n            uint8_t col[4] = {s[0][c]",
     "            (void)0;\n        for (int c = 0; c < 4; c++) {\n            uint8_t col[4] = {s[0][c]"),
    ("ctr_little_endian", "blk[12] = (uint8_t)(counter >> 24);", "blk[12] = (uint8_t)(counter);"),
    ("ctr_no_overflow_check", "> 0xFFFFFFFFull", "> 0xFFFFFFFFFFull"),
    ("le128_no_carry", "carry = sum >> 8;", "carry = 0;"),
    ("cbc_prev_block", "j->in + 16 * (i - 1);", "j->in + 16 * i;"),
    ("thread_chunks", "jobs[t].blk_end = n_blocks * (size_t)(t + 1) / (size_t)threads;",
     "jobs[t].blk_end = n_blocks * (size_t)(t + 1) / (size_t)threads - (t == 0);"),
]


@functools.lru_cache(maxsize=None)
def _source():
    with open(oracle.SOURCE) as f:
        return f.read()


QUICK = [functools.partial(P.pin_field, full=False), P.pin_field_order, P.pin_inverse, P.pin_sbox,
         P.pin_shift_rows_eq1, functools.partial(P.pin_mix_columns, n_random=50),
         functools.partial(P.pin_eq1_round, n=20), P.pin_lookup_count,
         functools.partial(P.pin_ttable_cipher, n_blocks=200),
         functools.partial(P.pin_round_trip, n_blocks=64), P.pin_key_schedule_prefix,
         P.pin_ctr_properties, P.pin_ctr_le128, P.pin_cbc, P.pin_sampled, P.pin_threads]
if openssl_ref.available():
    QUICK.append(functools.partial(P.pin_openssl, n_blocks=4))


def test_mutant_texts_apply():
    src = _source()
    for name, old, new in MUTANTS:
        assert src.count(old) == 1, f"mutant {name}: anchor text not found exactly once"


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    src = _source()
    assert src.count(old) == 1
    path = oracle.build_variant(src.replace(old, new), str(tmp_path), f"mutant_{name}")
    mutant = oracle.Oracle(path)
    failed = []
    for pin in QUICK:
        try:
            pin(mutant)
        except Exception as e:  # noqa: BLE001 - any failure counts as caught
            failed.append((getattr(pin, "func", pin).__name__, repr(e)[:80]))
            break
    assert failed, f"mutant {name} passed every pin"
