"""The CPU oracle against its pins (no GPU)."""
import pytest

from oracle_pins import all_pins

PINS = all_pins()


@pytest.mark.parametrize("name,fn", PINS, ids=[p[0] for p in PINS])
def test_pin(orc, name, fn):
    fn(orc)
