"""P3: one collision at one node, expanded by hand (Sec. 2, eqs. forcing, feq1-feq3, lbe).

Set-up: tau_A = tau_B = 1, G = 0.9, no walls, all populations at rest equilibrium.  Around the
node at x = 4 the densities are linear in x:  n_A(x) = 2.0 - 0.09 (x - 4), n_B = 0.06 + 0.09 (x - 4).
By hand:
  sum_i w_i n_B(x + c_i) c_i = (1/9 + 2/36) (n_B(5) - n_B(3)) e_x = (1/6)(0.18) e_x = 0.03 e_x
  a_A = F_A / n_A = -G * 0.03 = -0.027 e_x,  a_B = -G (1/6)(n_A(5) - n_A(3)) e_x = +0.027 e_x
  j = 0 at rest, so U = 0 and u_A^eq = tau a_A = (-0.027, 0), u_B^eq = (0.027, 0)
  tau = 1 means f* = f^eq(n, u^eq), e.g. f*_1^A = (2/9)(1 - 0.081 + 4.5*0.000729 - 1.5*0.000729)
"""
import numpy as np

import oracle

CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4

# The same expansion written out to ten digits.
EXPECT_A = [0.8879168889, 0.2047082222, 0.2219792222, 0.2407082222, 0.2219792222,
            0.0511770556, 0.0601770556, 0.0601770556, 0.0511770556]
EXPECT_B = [0.0266375067, 0.0072212467, 0.0066593767, 0.0061412467, 0.0066593767,
            0.0018053117, 0.0015353117, 0.0015353117, 0.0018053117]


def _setup():
    nx, ny = 9, 3
    x = np.arange(nx, dtype=float)
    nA = np.broadcast_to(2.0 - 0.09 * (x - 4), (ny, nx)).copy()
    nB = np.broadcast_to(0.06 + 0.09 * (x - 4), (ny, nx)).copy()
    o = oracle.Oracle(nx, ny, 0, 0, G=0.9, gw=(0.0, 0.0), tau=(1.0, 1.0))
    o.init(nA, nB)
    return o


def test_intermediates():
    m = _setup().macro()
    y, x = 1, 4
    assert abs(m["n"][0, y, x] - 2.0) < 1e-15 and abs(m["n"][1, y, x] - 0.06) < 1e-15
    assert np.all(np.abs(m["j"][:, :, y, x]) < 1e-15)
    assert abs(m["F"][0, 0, y, x] - 2.0 * -0.027) < 1e-14 and abs(m["F"][0, 1, y, x]) < 1e-15
    assert abs(m["F"][1, 0, y, x] - 0.06 * 0.027) < 1e-15
    assert abs(m["U"][0, y, x]) < 1e-15 and abs(m["U"][1, y, x]) < 1e-15
    assert abs(m["ueq"][0, 0, y, x] + 0.027) < 1e-14 and abs(m["ueq"][1, 0, y, x] - 0.027) < 1e-13


def test_post_collision_populations():
    o = _setup()
    o.step(1)
    f = o.populations()
    y, x = 1, 4
    # after streaming, f*_i(x) sits at x + c_i
    got = np.array([[f[k, i, (y + CY[i]) % 3, x + CX[i]] for i in range(9)] for k in range(2)])
    for k, (n, ux) in enumerate([(2.0, -0.027), (0.06, 0.027)]):
        hand = np.array([W[i] * n * (1 + 3 * CX[i] * ux + 4.5 * (CX[i] * ux) ** 2 - 1.5 * ux * ux)
                         for i in range(9)])
        np.testing.assert_allclose(got[k], hand, atol=1e-14)
    np.testing.assert_allclose(got[0], EXPECT_A, atol=1e-10)
    np.testing.assert_allclose(got[1], EXPECT_B, atol=1e-10)
    # mass is kept and the momentum gained equals the force, F_A = n_A a_A = -0.054
    assert abs(got[0].sum() - 2.0) < 1e-14
    assert abs(np.dot(CX, got[0]) + 0.054) < 1e-14


# ------------------------------------------------------------------------------ molecular masses
# P3 again with molecular masses m = (1, 1.5) (rho_k = m_k n_k, Sec. 2) and tau = (1, 0.8), the
# populations moving: f^A = f^eq(n_A(x), u = (0.02, 0)), f^B = f^eq(n_B(x), u = (-0.05, 0.01)),
# the same linear densities around x = 4.  By hand at x = 4:
#   j_A = (0.04, 0), j_B = (-0.003, 0.0006); rho_A = 2.0, rho_B = 0.09
#   F_A = -n_A G (0.03, 0) = (-0.054, 0);  F_B = -n_B G (-0.03, 0) = (0.00162, 0)
#   U = (m_A j_A / 1 + m_B j_B / 0.8) / (rho_A / 1 + rho_B / 0.8)
#     = (0.04 - 0.005625, 0.001125) / 2.1125 = (0.0162721893491, 0.000532544378698)
#   u_A^eq = U + 1.0 F_A / rho_A = U + (-0.027, 0)
#   u_B^eq = U + 0.8 F_B / rho_B = U + (0.0144, 0)
#   f*_i = f_i - (f_i - f_i^eq(n, u^eq)) / tau, evaluated to twelve digits with exact fractions.
# A mass factor dropped from U (n_k in place of rho_k) or from u^eq (F_k / n_k) moves every
# B population in the third decimal.
U_MASS = (0.016272189349112426, 0.0005325443786982248)
EXPECT_A_MASS = [0.888735062856, 0.215146977868, 0.222539078903, 0.229450725403, 0.221829019732,
                 0.053872716247, 0.057454366166, 0.057271138337, 0.053700914489]
EXPECT_B_MASS = [0.026645613327, 0.007694737435, 0.006623977576, 0.005661127968, 0.006697350357,
                 0.001916509188, 0.001403744285, 0.001426450017, 0.001930489847]


def _textbook_feq(n, ux, uy):
    return np.array([W[i] * n * (1 + 3 * (CX[i] * ux + CY[i] * uy) + 4.5 * (CX[i] * ux + CY[i] * uy) ** 2
                                 - 1.5 * (ux * ux + uy * uy)) for i in range(9)])


def _setup_mass():
    nx, ny = 9, 3
    f = np.zeros((2, 9, ny, nx))
    for x in range(nx):
        f[0, :, :, x] = _textbook_feq(2.0 - 0.09 * (x - 4), 0.02, 0.0)[:, None]
        f[1, :, :, x] = _textbook_feq(0.06 + 0.09 * (x - 4), -0.05, 0.01)[:, None]
    o = oracle.Oracle(nx, ny, 0, 0, G=0.9, gw=(0.0, 0.0), tau=(1.0, 0.8), mass=(1.0, 1.5))
    o.set_populations(f)
    return o, f


def test_intermediates_unequal_masses():
    o, _ = _setup_mass()
    m = o.macro()
    y, x = 1, 4
    assert abs(m["F"][0, 0, y, x] + 0.054) < 1e-14 and abs(m["F"][1, 0, y, x] - 0.00162) < 1e-15
    assert abs(m["U"][0, y, x] - U_MASS[0]) < 1e-15 and abs(m["U"][1, y, x] - U_MASS[1]) < 1e-15
    assert abs(m["ueq"][0, 0, y, x] - (U_MASS[0] - 0.027)) < 1e-14
    assert abs(m["ueq"][1, 0, y, x] - (U_MASS[0] + 0.0144)) < 1e-13
    assert abs(m["ueq"][1, 1, y, x] - U_MASS[1]) < 1e-15


def test_post_collision_unequal_masses():
    o, f0 = _setup_mass()
    o.step(1)
    f = o.populations()
    y, x = 1, 4
    got = np.array([[f[k, i, (y + CY[i]) % 3, x + CX[i]] for i in range(9)] for k in range(2)])
    np.testing.assert_allclose(got[0], EXPECT_A_MASS, atol=1e-11)
    np.testing.assert_allclose(got[1], EXPECT_B_MASS, atol=1e-11)
    # each component keeps its particle number; the mass-weighted momentum gained equals the
    # total force on the node, F_A + F_B = -0.05238
    assert abs(got[0].sum() - 2.0) < 1e-14 and abs(got[1].sum() - 0.06) < 1e-15
    fA, fB = f0[0, :, y, x], f0[1, :, y, x]
    dP = 1.0 * np.dot(CX, got[0] - fA) + 1.5 * np.dot(CX, got[1] - fB)
    assert abs(dP + 0.05238) < 1e-14


def test_init_takes_mass_densities():
    """scf/oracle init takes rho_k = m_k n_k (Sec. 2) and sets rest populations of n_k = rho_k / m_k."""
    rho_a = np.full((3, 5), 2.0)
    rho_b = np.full((3, 5), 0.09)
    o = oracle.Oracle(5, 3, 0, 0, tau=(1.0, 0.8), mass=(1.0, 1.5)).init(rho_a, rho_b)
    nA, nB = o.density()
    np.testing.assert_allclose(nA, 2.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(nB, 0.06, rtol=0, atol=1e-15)
    f = o.populations()
    np.testing.assert_allclose(f[1, :, 1, 2], _textbook_feq(0.06, 0.0, 0.0), rtol=0, atol=1e-16)
