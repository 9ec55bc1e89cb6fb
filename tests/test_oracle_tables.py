"""Pins for beta-bar (Eq. betaBar) and the integer acceptance table.

For p = 3/(m+3) the paper's weight (p/3)/(1-p) is exactly 1/m, so
A[Delta] = floor(2^32 / m^Delta) has an integer closed form (m = 17 at the
benchmark rate p = 0.15).
"""

import math

import numpy as np
import pytest

from oracle import tables


@pytest.mark.parametrize("m", [7, 9, 17, 37, 57])
def test_closed_form_table(m):
    p = 3.0 / (m + 3.0)
    got = tables.acceptance_table(tables.beta_bar(p))
    want = [(1 << 32) // m**d for d in range(1, 5)]
    assert got.tolist() == want


def test_p015_values():
    assert tables.tables(0.15, 1)[0].tolist() == [252645135, 14861478, 874204, 51423]
    assert math.isclose(tables.beta_bar(0.15), math.log(17.0), rel_tol=1e-15)


def test_ladder():
    b = tables.beta_bar(0.15)
    lad = tables.ladder(0.15, 20)
    assert len(lad) == 20 and lad[-1] == pytest.approx(b, rel=1e-15)
    assert all(lad[i] < lad[i + 1] for i in range(19))
    # beta_10 = beta_bar / 2: A[2] = floor(2^32 / 17) in closed form
    assert tables.acceptance_table(lad[9])[1] == (1 << 32) // 17
    assert tables.ladder(0.15, 1) == [b]


def test_monotone_and_limits():
    for p in (0.01, 0.05, 0.1, 0.15, 0.18, 0.5, 0.7):
        a = tables.acceptance_table(tables.beta_bar(p)).astype(np.int64)
        assert (np.diff(a) < 0).all() or (a == 0).all()
    # very cold: A[4] underflows to 0 (the move is never taken)
    assert tables.acceptance_table(40.0).tolist() == [0, 0, 0, 0]
    for bad in (0.0, -0.1, 0.75, 0.9, float("nan")):
        with pytest.raises(ValueError):
            tables.beta_bar(bad)


def test_error_threshold():
    assert tables.error_threshold(0.25) == 1 << 30
    assert tables.error_threshold(0.5) == 1 << 31
    assert tables.error_threshold(0.15) == math.floor(0.15 * 2**32)
