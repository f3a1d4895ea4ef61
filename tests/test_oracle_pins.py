"""CPU pins of the FP64 oracle (closed forms, brute force, invariants, finite differences)."""

import pytest

from tests import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=[p.__name__ for p in P.ALL_PINS])
def test_oracle_pin(oracle_lib, pin):
    pin()
