"""The CPU oracle against its pins (hand-worked fixtures, closed forms, brute
force, float64 bounds and invariants).  CPU only."""
import pytest

from oracle import oracle
from tests import pins


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.mark.parametrize("pin", pins.PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)
