"""The CPU oracle against its pins (exact mathematics and an independent
Philox implementation); see tests/pins.py for what each pin fixes."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.parametrize("name", list(pins.ALL_PINS))
def test_pin(orc, name):
    pins.ALL_PINS[name](orc)
