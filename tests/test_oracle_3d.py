"""Pins of the three-dimensional (D3Q19) oracle, independent of its code:

* the equilibrium's moments: sum f = n, sum c f = n u, sum c c f = n I / 3 + n u u;
* a state that does not depend on z evolves exactly as the two-dimensional model of Sec. 2 (the
  z-projection of the D3Q19 weights is the D2Q9 set with rest fraction 4/9), checked against the
  already-pinned 2-D oracle on the capillary;
* brute force on tiny boxes: forces summed over all node pairs by distance (1/18 at distance 1,
  1/36 at sqrt 2, minimum image), the textbook equilibrium and push streaming with reflection;
* mass conservation in a walled duct and momentum conservation without walls.
"""
import numpy as np
import pytest

import oracle
from oracle import CX3, CY3, CZ3
from paper_0807_0602_amd import inputs

C3 = np.stack([CX3, CY3, CZ3], axis=1)
W3 = np.where((C3 ** 2).sum(1) == 0, 1 / 3, np.where((C3 ** 2).sum(1) == 1, 1 / 18, 1 / 36))
OPP3 = [int(np.where((C3 == -C3[i]).all(axis=1))[0][0]) for i in range(19)]


@pytest.mark.parametrize("seed", range(4))
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    n = rng.uniform(0.05, 2.5)
    u = rng.uniform(-0.1, 0.1, 3)
    f = oracle.feq3(n, *u)
    assert f.sum() == pytest.approx(n, rel=1e-14)
    np.testing.assert_allclose(C3.T @ f, n * u, atol=1e-15)
    P = np.einsum("i,ia,ib->ab", f, C3, C3)
    np.testing.assert_allclose(P, n / 3 * np.eye(3) + n * np.outer(u, u), atol=2e-15)


def test_z_invariant_state_is_the_2d_model():
    case = inputs.capillary_small(seed=3)
    g, p = case.geom, case.params
    a2, b2 = case.fields()
    nz = 3
    o2 = oracle.Oracle.from_case(case).init(a2, b2).step(60)
    o3 = oracle.Oracle3(g.nx, g.ny, nz, g.x0, g.x1, walls_y=True, walls_z=False, G=p.G, gw=p.gw,
                        tau=p.tau).init(np.repeat(a2[None], nz, 0), np.repeat(b2[None], nz, 0)).step(60)
    rA, rB = o2.density()
    nA, nB = o3.density()
    for z in range(nz):
        np.testing.assert_allclose(nA[z], rA, rtol=0, atol=1e-12)
        np.testing.assert_allclose(nB[z], rB, rtol=0, atol=1e-12)
    obs2, obs3 = o2.observe(), o3.observe()
    assert abs(obs3["z"] - obs2["z"]) < 1e-9
    for k in range(2):
        assert obs3["mass"][k] == pytest.approx(nz * obs2["mass"][k], rel=1e-12)


def _min_image(d, n):
    d = d % n
    return d - n if d > n // 2 else d


def _brute_step3(f, solid, G, gw, tau):
    _, _, nz, ny, nx = f.shape
    n = f.sum(axis=1) * (~solid)[None]
    j = np.einsum("kizyx,id->kdzyx", f, C3)
    post = np.zeros_like(f)
    out = np.zeros_like(f)
    nodes = [(z, y, x) for z in range(nz) for y in range(ny) for x in range(nx)]
    for (z, y, x) in nodes:
        if solid[z, y, x]:
            continue
        F = np.zeros((2, 3))
        for (zp, yp, xp) in nodes:
            d = np.array([_min_image(xp - x, nx), _min_image(yp - y, ny), _min_image(zp - z, nz)])
            r2 = d @ d
            w = 1 / 18 if r2 == 1 else (1 / 36 if r2 == 2 else 0.0)
            if w == 0.0:
                continue
            for k in range(2):
                F[k] -= n[k, z, y, x] * w * (G * n[1 - k, zp, yp, xp] + gw[k] * float(solid[zp, yp, xp])) * d
        U = sum(j[k, :, z, y, x] / tau[k] for k in range(2)) / sum(n[k, z, y, x] / tau[k] for k in range(2))
        for k in range(2):
            u = U + tau[k] * F[k] / n[k, z, y, x]
            cu = C3 @ u
            fe = W3 * n[k, z, y, x] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u @ u))
            post[k, :, z, y, x] = f[k, :, z, y, x] - (f[k, :, z, y, x] - fe) / tau[k]
    for (z, y, x) in nodes:
        if solid[z, y, x]:
            continue
        for i in range(19):
            zt, yt, xt = (z + C3[i, 2]) % nz, (y + C3[i, 1]) % ny, (x + C3[i, 0]) % nx
            if solid[zt, yt, xt]:
                out[:, OPP3[i], z, y, x] = post[:, i, z, y, x]
            else:
                out[:, i, zt, yt, xt] = post[:, i, z, y, x]
    return out


@pytest.mark.parametrize("nx,ny,nz,x0,x1,wy,wz,tau,gw", [
    (4, 4, 3, 1, 3, True, False, (1.0, 1.0), (-0.2, 0.2)),
    (5, 4, 4, 0, 5, True, True, (0.8, 1.3), (0.3, -0.1)),
    (4, 3, 5, 2, 4, False, True, (1.4, 0.9), (-0.25, 0.0)),
])
def test_matches_pairwise_reference(nx, ny, nz, x0, x1, wy, wz, tau, gw):
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    G = 0.9
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inx = (X >= x0) & (X < x1)
    solid = inx & ((wy & ((Y == 0) | (Y == ny - 1))) | (wz & ((Z == 0) | (Z == nz - 1))))
    f = rng.uniform(0.01, 0.2, size=(2, 19, nz, ny, nx)) * (~solid)[None, None]
    o = oracle.Oracle3(nx, ny, nz, x0, x1, walls_y=wy, walls_z=wz, G=G, gw=gw, tau=tau)
    o.set_populations(f)
    ref = f.copy()
    for _ in range(2):
        o.step(1)
        ref = _brute_step3(ref, solid, G, gw, tau)
        np.testing.assert_allclose(o.populations(), ref, rtol=0, atol=1e-13)


def test_mass_in_a_duct_and_momentum_without_walls():
    nx, ny, nz = 40, 10, 8
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    liq = X < 12
    a = np.where(liq, 2.0, 0.06) + 1e-3 * inputs.uniform_pm1(7, 0, Y * nz + Z, X)
    b = np.where(liq, 0.06, 2.0) + 1e-3 * inputs.uniform_pm1(7, 1, Y * nz + Z, X)
    o = oracle.Oracle3(nx, ny, nz, 12, 32, walls_y=True, walls_z=True, G=0.9, gw=(-0.2, 0.2))
    o.init(a, b)
    m0 = o.observe()["mass"]
    o.step(200)
    m1 = o.observe()["mass"]
    for k in range(2):
        assert abs(m1[k] - m0[k]) / m0[k] <= 1e-12
    rng = np.random.default_rng(2)
    f = rng.uniform(0.02, 0.2, size=(2, 19, 6, 5, 7))
    o = oracle.Oracle3(7, 5, 6, 0, 0, walls_y=False, walls_z=False, G=0.9, tau=(1.0, 0.8))
    o.set_populations(f)
    p0 = np.einsum("kizyx,id->d", o.populations(), C3)
    assert np.abs(p0).max() > 0.05
    o.step(50)
    p1 = np.einsum("kizyx,id->d", o.populations(), C3)
    np.testing.assert_allclose(p1, p0, rtol=0, atol=1e-12)
