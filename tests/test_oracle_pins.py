"""The oracle against its pins (closed forms, invariants, quadrature and
printed numbers; see ``pin_suite.py``).  CPU only."""
import pytest

import pin_suite


@pytest.mark.parametrize("pin", pin_suite.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin(None)
