"""The oracle against the facts that pin it (see tests/oracle_pins.py)."""
import pytest

import oracle
from tests import oracle_pins


@pytest.mark.parametrize("check", oracle_pins.ALL_CHECKS, ids=lambda c: c.__name__)
def test_oracle_pin(check):
    check(oracle.lib())


def test_domain():
    import numpy as np
    F = oracle.boys_ld(np.array([np.nan, np.inf, -2.0]), 5)
    assert np.all(np.isnan(F[0])) and np.all(F[1] == 0) and np.all(np.isnan(F[2]))
    with pytest.raises(ValueError):
        oracle.boys([1.0], oracle.KMAX_LIMIT + 1)
