"""The CPU oracle against facts fixed outside it (see ``oracle_pins``)."""
import pytest

import oracle
import openssl_ref
import oracle_pins as P


@pytest.fixture(scope="module")
def o():
    return oracle.default()


@pytest.mark.parametrize("pin", [p for p in P.ALL_PINS if p is not P.pin_openssl],
                         ids=lambda p: p.__name__)
def test_pin(o, pin):
    pin(o)


@pytest.mark.skipif(not openssl_ref.available(), reason="system openssl not present")
def test_pin_openssl(o):
    P.pin_openssl(o)


def test_key_length_rejected(o):
    with pytest.raises(oracle.OracleError) as e:
        o.ecb_encrypt(bytes(15), bytes(16))
    assert e.value.status == oracle.EKEYLEN


def test_empty_inputs(o):
    assert o.ecb_encrypt(bytes(16), b"").size == 0
    assert o.ctr(bytes(16), bytes(12), 1, b"").size == 0
