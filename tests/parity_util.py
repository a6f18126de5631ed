"""Comparison helpers for the parity tests that never let a non-finite value pass.

Python's built-in max() keeps its first argument when a later one is NaN (NaN compares false),
so an accumulator such as `worst = max(worst, abs(a - b))` silently swallows a NaN on either
side.  Every parity comparison goes through these helpers instead:

* max_abs_diff: fields that must be finite on both sides (densities, populations); a non-finite
  value anywhere fails the test.
* front_diff: a front position (z, precursor) that may legitimately be absent (NaN) on both
  sides; NaN on one side only compares as an infinite difference.
"""
from __future__ import annotations

import math

import numpy as np


def max_abs_diff(*pairs) -> float:
    """Largest |a - b| over all (a, b) pairs of arrays; asserts that every value is finite."""
    worst = 0.0
    for i, (a, b) in enumerate(pairs):
        a = np.asarray(a, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        assert a.shape == b.shape, f"pair {i}: shapes {a.shape} and {b.shape}"
        assert np.isfinite(a).all(), f"pair {i}: non-finite value in the first field"
        assert np.isfinite(b).all(), f"pair {i}: non-finite value in the second field"
        if a.size:
            worst = max(worst, float(np.abs(a - b).max()))
    return worst


def front_diff(g: float, r: float) -> float:
    """|g - r| for front positions; 0 if both are absent (NaN), inf if only one is."""
    gn, rn = math.isnan(g), math.isnan(r)
    if gn and rn:
        return 0.0
    if gn or rn:
        return math.inf
    return abs(g - r)


def worst_of(values) -> float:
    """Largest of a sequence of differences; NaN anywhere gives NaN (which fails any <= check)."""
    v = np.asarray(list(values), dtype=np.float64)
    if v.size == 0:
        return 0.0
    return float(np.nan if np.isnan(v).any() else v.max())
