"""The parity helper itself (CPU): every slot of every query is checked."""
import numpy as np
import pytest

from gpu_util import assert_same


def _ref():
    oi = np.array([[0, 1, 2], [3, 4, -1], [5, 6, 7]], dtype=np.int64)
    od = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, np.inf], [6.0, 7.0, 8.0]])
    return oi, od


def test_identical_results_pass():
    oi, od = _ref()
    assert_same(oi.copy(), od.copy(), oi, od)
    # rows without a metric: (-1, NaN) on both sides
    gi = np.full((1, 3), -1)
    nan = np.full((1, 3), np.nan)
    assert_same(gi, nan, gi.copy(), nan.copy())


def test_index_mismatch_in_a_later_row_fails():
    oi, od = _ref()
    gi = oi.copy()
    gi[2, 1] = 9
    with pytest.raises(AssertionError):
        assert_same(gi, od, oi, od)


def test_distance_mismatch_in_the_second_row_fails():
    """The first row differs within the tolerance, the second beyond it:
    the second must still be caught."""
    oi, od = _ref()
    gd = od.copy()
    gd[0, 0] *= 1 + 1e-15
    gd[1, 1] *= 1 + 1e-9
    with pytest.raises(AssertionError):
        assert_same(oi, gd, oi, od)
    gd[1, 1] = od[1, 1]
    assert_same(oi, gd, oi, od)


def test_nan_against_a_number_fails():
    oi, od = _ref()
    gd = od.copy()
    gd[2, 2] = np.nan
    with pytest.raises(AssertionError):
        assert_same(oi, gd, oi, od)
    gd = od.copy()
    gd[1, 2] = 5.0  # finite where the oracle has an empty (+inf) slot
    with pytest.raises(AssertionError):
        assert_same(oi, gd, oi, od)
