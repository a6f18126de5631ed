"""The observables (mass, centre-line front z, precursor, health flag) on fields built by hand.

Populations are placed on the rest direction only, so n_k equals the chosen field exactly.
"""
import math

import numpy as np

import oracle


def _with_density(nx, ny, x0, x1, nA, nB):
    o = oracle.Oracle(nx, ny, x0, x1)
    f = np.zeros((2, 9, ny, nx))
    f[0, 0] = nA
    f[1, 0] = nB
    o.set_populations(f)
    return o


def test_front_and_precursor_by_hand():
    nx, ny, x0, x1 = 40, 8, 10, 30
    x = np.arange(nx, dtype=float)
    # phi = nA - nB crosses zero between x = 17 and 18 at 17.25 on the centre rows 3 and 4
    nA = np.broadcast_to(np.clip(2.0 - 0.5 * (x - 16.5), 0.06, 2.0), (ny, nx)).copy()
    nB = np.broadcast_to(np.clip(0.06 + 0.5 * (x - 16.5), 0.06, 2.0), (ny, nx)).copy()
    # wall rows 1 and ny-2: liquid reaches further (the film), n_A falls linearly 2 -> 0.06
    nA[1] = nA[ny - 2] = np.clip(2.0 - 0.1 * (x - 15.0), 0.06, 2.0)
    solid = np.zeros((ny, nx), bool); solid[0, x0:x1] = solid[ny - 1, x0:x1] = True
    nA[solid] = 0; nB[solid] = 0
    o = _with_density(nx, ny, x0, x1, nA, nB)
    obs = o.observe()
    # phi(x) = 1.94 - (x - 16.5) on the ramp: zero at x = 18.44
    assert abs(obs["z"] - (18.44 - x0)) < 1e-12
    # bulk n_A(xs = 5, centre) = 2.0, level 2/3: 2 - 0.1 (x - 15) = 2/3 at x = 28.333..
    assert abs(obs["precursor"] - (15 + (2 - 2 / 3) / 0.1 - x0)) < 1e-12
    assert obs["flags"] == 0
    assert abs(obs["mass"][0] - nA.sum()) < 1e-12 and abs(obs["mass"][1] - nB.sum()) < 1e-12


def test_missing_front_and_health_flags():
    nx, ny = 30, 6
    nA = np.full((ny, nx), 0.06); nB = np.full((ny, nx), 2.0)
    nA[2, 3] = -0.01        # negative density at a fluid node
    o = _with_density(nx, ny, 10, 20, nA, nB)
    obs = o.observe()
    assert math.isnan(obs["z"]) and math.isnan(obs["precursor"])
    assert obs["flags"] & 1 and obs["flags"] & 2
    nA[2, 3] = float("nan")
    assert _with_density(nx, ny, 10, 20, nA, nB).observe()["flags"] & 2
