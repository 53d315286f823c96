"""The oracle against closed forms, invariants, special cases and brute-force RK4."""
import pytest

from . import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin, oracle_lib):
    pin(oracle_lib)
