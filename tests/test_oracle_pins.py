"""The FP64 oracle against closed forms, special cases, invariants, brute force,
the paper's convergence statement and finite differences (see ``pins.py``)."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def lib():
    return oracle.load()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(lib, pin):
    pin(lib)
