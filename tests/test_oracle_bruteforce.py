"""P13: brute force on tiny boxes with an independent formulation of Sec. 2-3.

The reference below is written differently from the oracle on purpose:
  * forces sum over ALL pairs of nodes (x, x') with the paper's interaction matrix by
    distance: g for |x'-x| = 1, g/4 for |x'-x| = sqrt 2, 0 otherwise (g = G/9), using
    minimum-image displacements in the periodic box;
  * the equilibrium is the textbook D2Q9 form w_i n (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u);
  * streaming is a push with reflection: f*_i(x) goes to x + c_i, or back into the
    opposite direction at x when x + c_i is solid.
"""
import numpy as np
import pytest

import oracle

C = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
OPP = [int(np.where((C == -C[i]).all(axis=1))[0][0]) for i in range(9)]


def _min_image(d, n):
    d = d % n
    return d - n if d > n // 2 else d


def brute_step(f, solid, G, gw, tau):
    _, _, ny, nx = f.shape
    n = f.sum(axis=1) * (~solid)[None]
    j = np.einsum("kiyx,id->kdyx", f, C)
    g = G / 9.0
    out = np.zeros_like(f)
    post = np.zeros_like(f)
    nodes = [(y, x) for y in range(ny) for x in range(nx)]
    for (y, x) in nodes:
        if solid[y, x]:
            continue
        F = np.zeros((2, 2))
        for (yp, xp) in nodes:
            d = np.array([_min_image(xp - x, nx), _min_image(yp - y, ny)])
            r2 = d @ d
            Gd = g if r2 == 1 else (g / 4 if r2 == 2 else 0.0)
            if Gd == 0.0:
                continue
            for k in range(2):
                F[k] -= n[k, y, x] * Gd * n[1 - k, yp, xp] * d
                # wall: same matrix shape with g_kw rho_w in place of g, i.e. G_kw/9 and G_kw/36
                F[k] -= n[k, y, x] * gw[k] * (Gd / G) * (1.0 if solid[yp, xp] else 0.0) * d
        U = sum(j[k, :, y, x] / tau[k] for k in range(2)) / sum(n[k, y, x] / tau[k] for k in range(2))
        for k in range(2):
            u = U + tau[k] * F[k] / n[k, y, x]
            cu = C @ u
            fe = W * n[k, y, x] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u @ u))
            post[k, :, y, x] = f[k, :, y, x] - (f[k, :, y, x] - fe) / tau[k]
    for (y, x) in nodes:
        if solid[y, x]:
            continue
        for i in range(9):
            yt, xt = (y + C[i, 1]) % ny, (x + C[i, 0]) % nx
            if solid[yt, xt]:
                out[:, OPP[i], y, x] = post[:, i, y, x]
            else:
                out[:, i, yt, xt] = post[:, i, y, x]
    return out


@pytest.mark.parametrize("nx,ny,x0,x1,tau,gw", [
    (5, 4, 1, 3, (1.0, 1.0), (-0.2, 0.2)),
    (6, 5, 0, 6, (0.8, 1.3), (0.3, -0.1)),
    (7, 4, 2, 5, (1.7, 0.9), (-0.25, 0.0)),
    (5, 5, 0, 0, (1.2, 0.7), (0.0, 0.0)),
])
def test_matches_pairwise_reference(nx, ny, x0, x1, tau, gw):
    rng = np.random.default_rng(nx * 100 + ny)
    G = 0.9
    solid = np.zeros((ny, nx), dtype=bool)
    solid[0, x0:x1] = True
    solid[ny - 1, x0:x1] = True
    # random positive populations, including a non-zero momentum
    f = rng.uniform(0.01, 0.3, size=(2, 9, ny, nx)) * (~solid)[None, None]
    o = oracle.Oracle(nx, ny, x0, x1, G=G, gw=gw, tau=tau)
    o.set_populations(f)
    ref = f.copy()
    for _ in range(3):
        o.step(1)
        ref = brute_step(ref, solid, G, gw, tau)
        np.testing.assert_allclose(o.populations(), ref, rtol=0, atol=1e-13)


def test_init_is_rest_equilibrium():
    rng = np.random.default_rng(5)
    nA = rng.uniform(0.05, 2.1, size=(4, 6)); nB = rng.uniform(0.05, 2.1, size=(4, 6))
    o = oracle.Oracle(6, 4, 2, 4, alpha=(4 / 9, 4 / 9))
    o.init(nA, nB)
    f = o.populations()
    solid = np.zeros((4, 6), bool); solid[0, 2:4] = solid[3, 2:4] = True
    for k, nk in enumerate([nA, nB]):
        exp = W[:, None, None] * nk[None] * (~solid)[None]
        np.testing.assert_allclose(f[k], exp, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_general_mask_matches_pairwise_reference(seed):
    """A solid mask of arbitrary shape (isolated nodes, posts touching the box edge so that the
    periodic wrap meets a wall) in place of the wall rows."""
    rng = np.random.default_rng(40 + seed)
    nx, ny = 7, 6
    solid = rng.random((ny, nx)) < 0.22
    solid[:, 0] |= seed == 2          # a full solid column at the wrap
    G, gw, tau = 0.9, (-0.3 + 0.2 * seed, 0.25), (1.0 + 0.3 * seed, 0.8)
    f = rng.uniform(0.01, 0.3, size=(2, 9, ny, nx)) * (~solid)[None, None]
    o = oracle.Oracle(nx, ny, 0, 0, G=G, gw=gw, tau=tau, solid=solid)
    o.set_populations(f)
    ref = f.copy()
    for _ in range(3):
        o.step(1)
        ref = brute_step(ref, solid, G, gw, tau)
        np.testing.assert_allclose(o.populations(), ref, rtol=0, atol=1e-13)


def test_mask_of_the_rows_equals_the_rows():
    """A mask holding exactly the wall rows reproduces the row geometry bit for bit."""
    from paper_0807_0602_amd import inputs
    case = inputs.capillary_small(seed=2)
    g = case.geom
    a, b = case.fields()
    o1 = oracle.Oracle.from_case(case).init(a, b).step(60)
    o2 = oracle.Oracle(g.nx, g.ny, g.x0, g.x1, 0.9, case.params.gw, case.params.tau,
                       solid=g.solid_mask()).init(a, b).step(60)
    assert np.array_equal(o1.populations(), o2.populations())
    assert o1.observe() == o2.observe()
