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
