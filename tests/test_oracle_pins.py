"""The FP64 oracle against Philox answers, closed forms, limits, brute force
and distribution tests (CPU only)."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS + P.KD_PINS + P.BG_PINS, ids=lambda f: f.__name__)
def test_pin(oracle_lib, pin):
    pin()
