"""The comparison helpers of the parity tests reject a NaN on either side (CPU)."""
import math

import numpy as np
import pytest

from parity_util import front_diff, max_abs_diff, worst_of


def test_max_abs_diff_rejects_nan_on_either_side():
    a = np.zeros((3, 4))
    b = np.zeros((3, 4))
    b[1, 2] = np.nan
    with pytest.raises(AssertionError):
        max_abs_diff((a, a), (a, b))      # NaN in the second pair's second field
    with pytest.raises(AssertionError):
        max_abs_diff((b, a))
    with pytest.raises(AssertionError):
        max_abs_diff((a, np.full((3, 4), np.inf)))
    c = a.copy()
    c[0, 0] = 3e-6
    assert max_abs_diff((a, a), (a, c)) == pytest.approx(3e-6)


def test_python_max_would_have_hidden_the_nan():
    # the hole the helpers close: max(finite, nan) keeps the finite value
    assert max(0.1, float("nan")) == 0.1


def test_front_diff():
    assert front_diff(float("nan"), float("nan")) == 0.0
    assert front_diff(1.0, float("nan")) == math.inf
    assert front_diff(float("nan"), 1.0) == math.inf
    assert front_diff(2.0, 1.75) == 0.25
    assert not (max(0.0, front_diff(1.0, float("nan"))) <= 0.5)


def test_worst_of():
    assert worst_of([]) == 0.0
    assert worst_of([0.1, 0.3]) == 0.3
    assert math.isnan(worst_of([0.1, float("nan"), 0.2]))
