"""Physics of the capillary on the GPU at the 4096 x 202 channel size (H = 200, capillary length
3072), against the front equation of Sec. 2.1 (eq. GWE) and its drag-corrected, inertia-free limit

    (mu_l - mu_g)(z^2 - z0^2)/2 + mu_g L (z - z0) = gamma H cos(theta) (t - t0) / 6.

gamma cos(theta) is measured independently from a static meniscus at the same parameters
(Delta p = 2 gamma cos / H), and mu_l, mu_g from the phase compositions inside the channel
(mu = sum_k rho_k nu_k, Sec. 2).  The late-window fit must be linear (R^2 >= 0.9995) with a slope
between 0.70 and 1.05 of the static prediction: a moving contact line has a larger (dynamic)
angle than the static one (measured on the 200 x 24 capillary: cos 0.345 moving vs 0.475 static),
which lowers the slope.  The precursor film stays ahead of the centre-line front while the
reservoir lasts.
"""
import sys

import numpy as np
import pytest

from oracle import front, physics
from paper_0807_0602_amd import inputs

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def scf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0807_0602_amd import scf as S
    return S


def _static_gamma_cos(S, tau, gw, H=200, nx=1024, steps=120_000):
    g = inputs.Geometry(nx, H + 2, 0, nx)
    a, b = inputs.plug_fields(g, nx // 4, 3 * nx // 4)
    ch = S.Channel(g, inputs.Params(G=0.9, gw=gw, tau=tau), a, b)
    ch.step(steps)
    nA, nB = ch.density()
    p = physics.pressure(nA, nB)
    rows = slice(H // 4 + 10, 3 * H // 4 - 8)
    p_liq = p[rows, nx // 2 - 20:nx // 2 + 20].mean()
    p_gas = np.concatenate([p[rows, :40], p[rows, nx - 40:]], axis=1).mean()
    ch.close()
    return H * (p_gas - p_liq) / 2.0


@pytest.mark.parametrize("tau", [(1.0, 1.0), (1.25, 1.0)])
def test_drag_corrected_front_law(scf, tau):
    case = inputs.with_params(inputs.capillary_washburn(seed=1), tau=tau)
    g = case.geom
    H, Lc = g.ny - 2, g.x1 - g.x0
    _say(f"case: {case.name} tau={tau}, 150000 steps")
    ch = scf.Channel.from_case(case)
    ts, zs, ps, fl = [], [], [], []
    for t in range(0, 150_001, 1000):
        if t:
            ch.step(1000)
        o = ch.observe()
        ts.append(t); zs.append(o["z"]); ps.append(o["precursor"]); fl.append(o["flags"])
        assert not o["flags"] & 2
    ts, zs, ps, fl = np.array(ts, float), np.array(zs), np.array(ps), np.array(fl)
    nA, nB = ch.density()
    yc = g.ny // 2
    zl = zs[-1]
    xl = int(g.x0 + 0.5 * zl)
    xg = int(g.x0 + zl + 0.5 * (Lc - zl))
    nu = [physics.kinematic_viscosity(t_) for t_ in tau]
    mu_l = nA[yc, xl] * nu[0] + nB[yc, xl] * nu[1]
    mu_g = nA[yc, xg] * nu[0] + nB[yc, xg] * nu[1]
    gcos = _static_gamma_cos(scf, tau, case.params.gw, H)
    m = ts >= 60_000
    z0 = zs[m][0]
    lhs = front.drag_corrected_lhs(zs[m], z0, mu_l, mu_g, Lc)
    coef = np.polyfit(ts[m], lhs, 1)
    r2 = 1.0 - np.sum((lhs - np.polyval(coef, ts[m])) ** 2) / np.sum((lhs - lhs.mean()) ** 2)
    pred = gcos * H / 6.0
    _say(f"  mu_l={mu_l:.4f} mu_g={mu_g:.4f} gamma cos={gcos:.4f} slope={coef[0]:.4f} pred={pred:.4f} "
         f"ratio={coef[0] / pred:.3f} R2={r2:.6f} z(150k)={zl:.1f}")
    assert r2 >= 0.9995
    assert 0.70 <= coef[0] / pred <= 1.05
    # the precursor film (wall rows, n_A above a third of the reservoir's bulk value, read at
    # the reservoir centre x0/2) leads the centre-line front while that reading is bulk liquid:
    # the channel draws the reservoir's far interface towards its centre, which it reaches once
    # about x0/2 * ny nodes of liquid (z ~ x0/2 * ny / H) have entered, so only fronts below 70 %
    # of that are used.  In this partial-wetting, equal-viscosity channel the lead stays nearly
    # constant, so it shrinks relative to the distance filled.
    z_res = 0.7 * (g.x0 / 2) * g.ny / H
    late = (ts >= 40_000) & np.isfinite(ps) & (fl == 0) & (zs > 0) & (zs < z_res)
    assert late.sum() >= 40
    d = ps[late] - zs[late]
    _say(f"  precursor lead {d[0]:.2f} -> {d[-1]:.2f} lu while z {zs[late][0]:.1f} -> {zs[late][-1]:.1f}")
    assert np.all(d > 0)
    assert d[-1] / zs[late][-1] < 0.5 * d[0] / zs[late][0]
