"""The FP64 oracle against its pins (see oracle_pins.py for what each pins)."""
import pytest

from oracle.oracle import load
import oracle_pins


@pytest.fixture(scope="module")
def orc():
    return load()


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)
