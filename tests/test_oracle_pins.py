"""The CPU oracle checked against closed forms, library routines, textbook
identities, exact enumeration and sampling statistics (no GPU needed)."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin()
