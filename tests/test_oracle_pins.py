"""The CPU oracle against the paper's printed values, closed forms, invariants,
brute force and identities (the pins are defined in oracle_pins.py)."""
import pytest

import oracle
from oracle_pins import ALL_PINS


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(oracle._ORACLE)
