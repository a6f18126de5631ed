"""Invariants the paper's set-up fixes (Sec. 2-3).

P4: per-component mass is conserved (periodic box, bounce-back walls).
P5: with no walls the total momentum sum_k m_k sum_i c_i f_i is conserved, because the pair
    force of eq. forcing is antisymmetric in (x, x') and the common velocity U conserves
    momentum at collision (also with unequal molecular masses m_k).
P6: the capillary is mirror-symmetric about its centre line, so is a noise-free solution.
Translation: a periodic shift of a wall-free initial state shifts the solution exactly.
"""
import numpy as np

import oracle
from paper_0807_0602_amd import inputs

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def test_mass_conservation_capillary():
    case = inputs.capillary_small(seed=1)
    o = oracle.Oracle.from_case(case).init(*case.fields())
    m0 = o.observe()["mass"]
    o.step(2000)
    m1 = o.observe()["mass"]
    for k in range(2):
        assert abs(m1[k] - m0[k]) / m0[k] <= 1e-12


def test_mass_conservation_rough_capillary():
    """Bounce-back conserves mass for any solid shape (rough walls and a post)."""
    case = inputs.capillary_rough(seed=1)
    o = oracle.Oracle.from_case(case).init(*case.fields())
    m0 = o.observe()["mass"]
    o.step(1000)
    obs = o.observe()
    for k in range(2):
        assert abs(obs["mass"][k] - m0[k]) / m0[k] <= 1e-12
    assert obs["flags"] == 0


def test_momentum_conservation_without_walls():
    rng = np.random.default_rng(11)
    nx, ny = 24, 16
    f = rng.uniform(0.02, 0.25, size=(2, 9, ny, nx))
    o = oracle.Oracle(nx, ny, 0, 0, G=0.9, tau=(1.0, 0.8))
    o.set_populations(f)

    def momentum():
        g = o.populations()
        return np.array([np.einsum("kiyx,i->", g, CX), np.einsum("kiyx,i->", g, CY)])

    p0 = momentum()
    assert np.abs(p0).max() > 0.1
    for _ in range(4):
        o.step(50)
        np.testing.assert_allclose(momentum(), p0, rtol=0, atol=1e-12)


def test_mass_weighted_momentum_conservation_unequal_masses():
    """P5 with molecular masses m = (1, 1.5) and tau = (1, 0.8): rho_k u_k = m_k j_k, and the
    collision conserves sum_k m_k j_k up to the total force, whose sum over a wall-free box
    vanishes.  A mass factor dropped from the common velocity U or from u^eq = U + tau F / rho
    breaks the conservation; the unweighted sum sum_k j_k is not conserved."""
    rng = np.random.default_rng(12)
    nx, ny = 24, 16
    m = (1.0, 1.5)
    f = rng.uniform(0.02, 0.25, size=(2, 9, ny, nx))
    o = oracle.Oracle(nx, ny, 0, 0, G=0.9, tau=(1.0, 0.8), alpha=(4 / 9, 0.6), mass=m)
    o.set_populations(f)

    def momenta():
        g = o.populations()
        jk = np.array([[np.einsum("iyx,i->", g[k], CX), np.einsum("iyx,i->", g[k], CY)] for k in range(2)])
        return m[0] * jk[0] + m[1] * jk[1], jk[0] + jk[1]

    p0, q0 = momenta()
    assert np.abs(p0).max() > 0.1
    drift = 0.0
    for _ in range(4):
        o.step(50)
        p, q = momenta()
        np.testing.assert_allclose(p, p0, rtol=0, atol=1e-12)
        drift = max(drift, float(np.abs(q - q0).max()))
    assert drift > 1e-4           # the unweighted momentum does move: the masses matter


def test_mirror_symmetry_capillary():
    case = inputs.capillary_small(seed=1)
    case = inputs.Case(case.geom, case.params, noise=0.0)
    o = oracle.Oracle.from_case(case).init(*case.fields())
    o.step(500)
    nA, nB = o.density()
    assert np.abs(nA - nA[::-1]).max() <= 1e-13
    assert np.abs(nB - nB[::-1]).max() <= 1e-13
    assert np.abs(nA - 2.0).max() > 0.5   # the front did move / an interface exists


def test_translation_invariance():
    rng = np.random.default_rng(3)
    nx, ny = 20, 12
    nA = rng.uniform(0.05, 2.0, size=(ny, nx))
    nB = rng.uniform(0.05, 2.0, size=(ny, nx))
    a = oracle.Oracle(nx, ny, tau=(1.0, 0.9)).init(nA, nB).step(30)
    sx, sy = 7, 5
    b = oracle.Oracle(nx, ny, tau=(1.0, 0.9)).init(np.roll(nA, (sy, sx), axis=(0, 1)),
                                                   np.roll(nB, (sy, sx), axis=(0, 1))).step(30)
    fa = np.roll(a.populations(), (sy, sx), axis=(2, 3))
    assert np.array_equal(fa, b.populations())


def test_thread_count_does_not_change_results():
    case = inputs.capillary_small(seed=2)
    oracle.set_threads(1)
    a = oracle.Oracle.from_case(case).init(*case.fields()).step(40).populations()
    oracle.set_threads(4)
    b = oracle.Oracle.from_case(case).init(*case.fields()).step(40).populations()
    oracle.set_threads(8)
    assert np.array_equal(a, b)


def test_window_light_cone():
    """A window with clamped x-edges agrees exactly with the full box at distance > 2T from
    its edges after T steps: each step couples nodes at most two links apart."""
    case = inputs.capillary_small(seed=4)
    T = 10
    full = oracle.Oracle.from_case(case).init(*case.fields()).step(T)
    xa, w = 120, 61          # window [120, 181) straddles the channel end at x = 150
    win = oracle.Oracle.from_case(case, periodic_x=False, x_offset=xa, width=w)
    win.init(*case.fields(xa, xa + w)).step(T)
    inner = slice(2 * T, w - 2 * T)
    np.testing.assert_array_equal(win.populations()[..., inner],
                                  full.populations()[..., xa:xa + w][..., inner])
