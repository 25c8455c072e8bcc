"""The CPU oracle against facts it does not produce itself (no GPU)."""
import pytest

import oracle
from oracle_pins import PINS


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_pin(pin):
    pin(oracle.default())


def test_oracle_rejects_bad_dim():
    import numpy as np
    with pytest.raises(ValueError):
        oracle.flux(4, 1.4, np.ones((6, 3)))
    with pytest.raises(ValueError):
        oracle.cons2char(2, 2, 1.4, np.ones((4, 3)))
