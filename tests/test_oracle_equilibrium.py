"""Pins of the equilibrium, eqs. feq1-feq3 (Sec. 2).

P1: its moments are fixed by the text: sum_i f_i = n, sum_i c_i f_i = n u and
    sum_i c_ia c_ib f_i = n cs^2 delta_ab + n u_a u_b with cs^2 = 3 (1 - alpha) / 5.
P2: at alpha = 4/9 it is the textbook D2Q9 equilibrium w_i n (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u)
    with w = 4/9, 1/9, 1/36.
"""
import numpy as np
import pytest

import oracle

# velocities by the paper's definition (cos, sin of the listed angles), built independently
C = np.array([[0, 0]] + [[round(np.cos(k * np.pi / 2)), round(np.sin(k * np.pi / 2))] for k in range(4)]
             + [[round(np.sqrt(2) * np.cos(k * np.pi / 2 + np.pi / 4)),
                 round(np.sqrt(2) * np.sin(k * np.pi / 2 + np.pi / 4))] for k in range(4)], dtype=float)


@pytest.mark.parametrize("alpha", [4.0 / 9.0, 0.0, 0.2, 0.8, 0.998])
@pytest.mark.parametrize("n,ux,uy", [(1.0, 0.0, 0.0), (2.0, 0.05, -0.02), (0.06, -0.1, 0.07), (0.34, 0.0, 0.12)])
def test_moments(alpha, n, ux, uy):
    f = oracle.feq(n, ux, uy, alpha)
    u = np.array([ux, uy])
    cs2 = 3.0 * (1.0 - alpha) / 5.0
    assert abs(f.sum() - n) <= 1e-15 * max(1.0, n)
    np.testing.assert_allclose(C.T @ f, n * u, atol=1e-15)
    P = np.einsum("ia,ib,i->ab", C, C, f)
    np.testing.assert_allclose(P, n * cs2 * np.eye(2) + n * np.outer(u, u), atol=2e-15)


def test_textbook_d2q9_at_four_ninths():
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    rng = np.random.default_rng(0)
    for _ in range(50):
        n = rng.uniform(0.01, 3.0)
        u = rng.uniform(-0.15, 0.15, size=2)
        cu = C @ u
        ref = w * n * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u @ u))
        np.testing.assert_allclose(oracle.feq(n, u[0], u[1], 4.0 / 9.0), ref, rtol=0, atol=1e-15)


def test_velocity_set_numbering():
    # opposite pairs 1-3, 2-4, 5-7, 6-8 and the lattice of unit and diagonal links
    assert np.array_equal(C[1], -C[3]) and np.array_equal(C[2], -C[4])
    assert np.array_equal(C[5], -C[7]) and np.array_equal(C[6], -C[8])
    assert np.array_equal(C[5], [1, 1]) and np.array_equal(C[6], [-1, 1])
