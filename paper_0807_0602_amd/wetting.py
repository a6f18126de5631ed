"""Wettability calibration on the GPU: the a-posteriori contact angle of Sec. 2.

The wall couplings G_kw of eq. forcingw fix the contact angle only indirectly, so the paper
measures it after the fact.  This module measures it on batches of static configurations that
the batched LBM advances together (one launch per step for the whole batch), with two
independent estimators:

* static meniscus: a liquid plug in a fully walled channel of height H.  At rest each meniscus is
  a circular arc of radius H / (2 cos theta), so the gas-liquid pressure jump is
  Delta p = p_gas - p_liq = 2 gamma cos(theta) / H (Young-Laplace in 2-D), with the surface
  tension gamma from Laplace's law Delta p = gamma / R on free droplets;
* sessile droplet: a drop of A resting on a wall.  A circle fitted to its interface (the
  n_A = n_B contour away from the wall) meets the wall plane - half a node inside the solid row,
  where half-way bounce-back puts it - at the contact angle: cos(theta) = (y_wall - y_c) / R.

The pressure is the model's equation of state with the force weights of the build (reading of
Sec. 2): p = sum_k m_k n_k c_k^2 + (G/3) n_A n_B with c_k^2 = 3 (1 - alpha_k) / 5, the second
moment of eqs. feq1-feq3; at alpha = 4/9 and m = 1 it is (n_A + n_B)/3 + (G/3) n_A n_B.

`contact_angle_map` tabulates both estimators over wall couplings and relaxation-time pairs;
`match_coupling` inverts a table, e.g. to find the repulsive gas coupling that gives the same
angle as a given attractive liquid coupling (the two wetting routes the paper compares in
Sec. 3).  Everything runs through the C ABI; the host only averages and fits the returned
density fields.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import inputs
from .inputs import Case, Geometry, Params
from .scf import Batch

Pair = Tuple[float, float]


def eos_pressure(nA: np.ndarray, nB: np.ndarray, G: float, alpha: Pair = (4.0 / 9.0, 4.0 / 9.0),
                 mass: Pair = (1.0, 1.0)) -> np.ndarray:
    """Pressure of the binary mixture: sum_k m_k n_k 3 (1 - alpha_k)/5 + (G/3) n_A n_B."""
    cA = 3.0 * (1.0 - alpha[0]) / 5.0
    cB = 3.0 * (1.0 - alpha[1]) / 5.0
    return mass[0] * cA * nA + mass[1] * cB * nB + (G / 3.0) * nA * nB


def _run(cases: Sequence[Case], fields, steps: int, fuse: int = 2):
    b = Batch(cases, sample_every=max(1, steps), max_samples=2, fields=fields)
    b.set_tile(128, 16, graph_steps=100, order=1, fuse=fuse)
    b.step(steps)
    recs, _ = b.observe(allow_unstable=True)
    out = []
    for c in range(len(cases)):
        nA, nB = b.density(c)
        flags = recs[c][-1]["flags"] if recs[c] else 0
        out.append((nA, nB, flags))
    b.close()
    return out


# ------------------------------------------------------------------------------ surface tension
def laplace_tension(tau: Pair = (1.0, 1.0), G: float = 0.9, radii: Sequence[float] = (10, 14, 18, 22),
                    n: int = 96, steps: int = 8000, alpha: Pair = (4.0 / 9.0, 4.0 / 9.0),
                    mass: Pair = (1.0, 1.0), rho: Pair = (2.0, 0.06), gas: Optional[Pair] = None) -> Dict:
    """gamma from Laplace's law on free droplets of A in periodic n x n boxes: least-squares
    fit of Delta p = p_in - p_out against 1/R, R from the droplet area (nodes with
    n_A > n_B).  `rho`: initial (majority, minority) densities of the drop, `gas`: initial
    (n_A, n_B) around it.  Returns gamma, the intercept, the per-droplet data and the smallest
    density seen, overall and per droplet (slightly negative minority densities occur with unequal
    sound speeds)."""
    geom = Geometry(n, n, 0, 0)
    prm = Params(G=G, gw=(0.0, 0.0), tau=tuple(tau), alpha=tuple(alpha), mass=tuple(mass))
    cases = [Case(geom, prm, noise=0.0, name=f"droplet_R{R}") for R in radii]
    fields = [inputs.droplet_fields(n, R, rho_liq=rho[0], rho_min=rho[1], gas=gas) for R in radii]
    res = _run(cases, fields, steps)
    dps, Rs = [], []
    c = (n - 1) / 2.0
    Y, X = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    r = np.hypot(X - c, Y - c)
    min_density = np.inf
    mins = []
    for (nA, nB, flags), R0 in zip(res, radii):
        if not (np.isfinite(nA).all() and np.isfinite(nB).all()):
            raise RuntimeError(f"droplet R = {R0} went unstable (non-finite density); start closer "
                               "to the coexisting compositions or change tau")
        mins.append(min(float(nA.min()), float(nB.min())))
        min_density = min(min_density, mins[-1])
        p = eos_pressure(nA, nB, G, alpha, mass)
        R = np.sqrt(np.count_nonzero(nA > nB) / np.pi)
        p_in = p[r < 0.5 * R].mean()
        p_out = p[r > R + 0.35 * (n / 2 - R)].mean()
        dps.append(p_in - p_out)
        Rs.append(R)
    A = np.stack([1.0 / np.asarray(Rs), np.ones(len(Rs))], axis=1)
    (gamma, icpt), *_ = np.linalg.lstsq(A, np.asarray(dps), rcond=None)
    return {"gamma": float(gamma), "intercept": float(icpt), "R": Rs, "dp": dps,
            "min_density": min_density, "min_densities": mins}


# ------------------------------------------------------------------------------ estimators
@dataclass(frozen=True)
class WallCase:
    gw: Pair
    tau: Pair = (1.0, 1.0)
    G: float = 0.9
    alpha: Pair = (4.0 / 9.0, 4.0 / 9.0)
    mass: Pair = (1.0, 1.0)

    def params(self) -> Params:
        return Params(G=self.G, gw=self.gw, tau=self.tau, alpha=self.alpha, mass=self.mass)


def meniscus_cos(cases: Sequence[WallCase], gamma: float, H: int = 40, L: int = 320,
                 steps: int = 30000, rho: Pair = (2.0, 0.06), gas: Optional[Pair] = None) -> List[Dict]:
    """Static-meniscus estimator: a plug of A over the middle half of a fully walled periodic
    channel (L x H fluid rows); cos(theta) = H (p_gas - p_liq) / (2 gamma), pressures averaged
    over the middle of the plug and of the gas, away from walls and menisci."""
    geom = Geometry(L, H + 2, 0, L)
    cs = [Case(geom, w.params(), noise=0.0) for w in cases]
    fields = [inputs.plug_fields(geom, L // 4, 3 * L // 4, rho_liq=rho[0], rho_min=rho[1], gas=gas)
              for _ in cases]
    res = _run(cs, fields, steps)
    rows = slice(1 + H // 4, 1 + 3 * H // 4)
    q = L // 16
    out = []
    for w, (nA, nB, flags) in zip(cases, res):
        p = eos_pressure(nA, nB, w.G, w.alpha, w.mass)
        p_liq = p[rows, L // 2 - q:L // 2 + q].mean()
        p_gas = np.concatenate([p[rows, :q], p[rows, L - q:]], axis=1).mean()
        dp = p_gas - p_liq
        out.append({"gw": w.gw, "tau": w.tau, "dp": float(dp), "cos": float(H * dp / (2.0 * gamma)),
                    "flags": int(flags)})
    return out


def _contour_points(phi: np.ndarray, y_min: int) -> np.ndarray:
    """Points where phi changes sign between neighbouring nodes (along x and along y), linearly
    interpolated, for rows / node pairs at y >= y_min."""
    pts = []
    ny, nx = phi.shape
    for y in range(y_min, ny - 1):
        a, b = phi[y, :-1], phi[y, 1:]
        for x in np.nonzero((a > 0) != (b > 0))[0]:
            pts.append((x + a[x] / (a[x] - b[x]), y))
    for y in range(y_min, ny - 2):
        a, b = phi[y, :], phi[y + 1, :]
        for x in np.nonzero((a > 0) != (b > 0))[0]:
            pts.append((x, y + a[x] / (a[x] - b[x])))
    return np.asarray(pts, dtype=np.float64)


def fit_circle(pts: np.ndarray) -> Tuple[float, float, float]:
    """Algebraic least-squares circle x^2 + y^2 + D x + E y + F = 0 -> (xc, yc, R)."""
    x, y = pts[:, 0], pts[:, 1]
    A = np.stack([x, y, np.ones_like(x)], axis=1)
    (D, E, F), *_ = np.linalg.lstsq(A, -(x * x + y * y), rcond=None)
    xc, yc = -D / 2.0, -E / 2.0
    return float(xc), float(yc), float(np.sqrt(xc * xc + yc * yc - F))


def meniscus_radius(nA: np.ndarray, nB: np.ndarray, x_front: float, H: int, skip: int = 0) -> Dict:
    """Radius of curvature of a meniscus spanning a channel of H fluid rows (rows 1..H, walls on
    rows 0 and H + 1): a circle fitted to the n_A = n_B contour points in the columns from
    x_front - 4 to x_front + H (the meniscus and its contact-line region, x_front the centre-line
    front) and the rows at least `skip` nodes from the wall rows.  Across a 2-D meniscus the
    pressure jumps by gamma / R (Laplace), i.e. 2 gamma cos(theta) / H with cos(theta) = H / (2 R)
    the apparent contact angle: the capillary pressure that drives the filling, moving or at rest."""
    phi = np.asarray(nA, dtype=np.float64) - np.asarray(nB, dtype=np.float64)
    x_lo = max(int(np.floor(x_front)) - 4, 0)
    x_hi = min(int(np.ceil(x_front)) + H, phi.shape[1])
    sub_ = phi[:H + 2, x_lo:x_hi].copy()
    sub_[0, :] = sub_[H + 1, :] = np.nan          # wall rows hold no fluid
    pts = _contour_points(np.nan_to_num(sub_, nan=0.0), 1 + skip)
    if len(pts):
        pts = pts[(pts[:, 1] >= 1 + skip) & (pts[:, 1] <= H - skip)]
    if len(pts) < 8:
        return {"R": float("nan"), "npts": int(len(pts))}
    xc, yc, R = fit_circle(pts)
    return {"R": R, "xc": xc + x_lo, "yc": yc, "npts": int(len(pts)),
            "cos": float(H / (2.0 * R)) if R > 0 else float("nan")}


def sessile_cos(cases: Sequence[WallCase], R: float = 24.0, nx: int = 160, ny: int = 72,
                steps: int = 30000, skip: int = 4, rho: Pair = (2.0, 0.06),
                gas: Optional[Pair] = None) -> List[Dict]:
    """Sessile-droplet estimator: a half-disc of A of radius R on the bottom wall of a fully
    walled channel (periodic in x), relaxed for `steps`; a circle fitted to the interface points
    at least `skip` nodes above the wall gives cos(theta) = (0.5 - y_c) / R_fit."""
    geom = Geometry(nx, ny, 0, nx)
    cs = [Case(geom, w.params(), noise=0.0) for w in cases]
    fields = [inputs.sessile_fields(geom, (nx - 1) / 2.0, R, rho_liq=rho[0], rho_min=rho[1], gas=gas)
              for _ in cases]
    res = _run(cs, fields, steps)
    out = []
    for w, (nA, nB, flags) in zip(cases, res):
        phi = nA - nB
        phi[0, :] = phi[-1, :] = -1.0      # solid rows count as outside the drop
        pts = _contour_points(phi, 1 + skip)
        # keep the droplet's own contour: points closer to the drop centre than to the box edge
        pts = pts[np.abs(pts[:, 0] - (nx - 1) / 2.0) < nx / 2.0 - 4] if len(pts) else pts
        if len(pts) < 8:
            out.append({"gw": w.gw, "tau": w.tau, "cos": float("nan"), "flags": int(flags)})
            continue
        xc, yc, Rf = fit_circle(pts)
        cos = (0.5 - yc) / Rf
        out.append({"gw": w.gw, "tau": w.tau, "cos": float(np.clip(cos, -1.0, 1.0)),
                    "xc": xc, "yc": yc, "R": Rf, "npts": int(len(pts)), "flags": int(flags)})
    return out


def contact_angle_map(gws: Sequence[Pair], taus: Sequence[Pair] = ((1.0, 1.0),), G: float = 0.9,
                      H: int = 40, steps: int = 30000, gammas: Optional[Dict[Pair, float]] = None) -> Dict:
    """theta(G_w, tau pair) from both estimators.  Returns a dict with the grid, gamma per tau
    pair, and arrays cos_meniscus, cos_sessile, theta_meniscus_deg, theta_sessile_deg of shape
    (len(taus), len(gws))."""
    cases = [WallCase(tuple(gw), tuple(t), G) for t in taus for gw in gws]
    if gammas is None:
        gammas = {tuple(t): laplace_tension(tuple(t), G)["gamma"] for t in taus}
    men: List[Dict] = []
    for t in taus:
        men += meniscus_cos([c for c in cases if c.tau == tuple(t)], gammas[tuple(t)], H=H, steps=steps)
    ses = sessile_cos(cases, steps=steps)
    shape = (len(taus), len(gws))
    cm = np.array([m["cos"] for m in men]).reshape(shape)
    cs = np.array([s["cos"] for s in ses]).reshape(shape)
    return {"gws": [tuple(g) for g in gws], "taus": [tuple(t) for t in taus], "gammas": gammas,
            "cos_meniscus": cm, "cos_sessile": cs,
            "theta_meniscus_deg": np.degrees(np.arccos(np.clip(cm, -1, 1))),
            "theta_sessile_deg": np.degrees(np.arccos(np.clip(cs, -1, 1))),
            "flags": np.array([m["flags"] | s["flags"] for m, s in zip(men, ses)]).reshape(shape)}


def match_coupling(values: Sequence[float], cos_values: Sequence[float], target_cos: float) -> float:
    """The coupling at which the tabulated cos(theta) reaches target_cos, by linear
    interpolation between the two bracketing table entries (values sorted ascending)."""
    v = np.asarray(values, dtype=np.float64)
    c = np.asarray(cos_values, dtype=np.float64)
    for i in range(len(v) - 1):
        lo, hi = c[i], c[i + 1]
        if (lo - target_cos) * (hi - target_cos) <= 0 and lo != hi:
            return float(v[i] + (target_cos - lo) * (v[i + 1] - v[i]) / (hi - lo))
    raise ValueError("target cos(theta) outside the tabulated range")


# ------------------------------------------------------------------------------ the two routes
def equivalent_couplings(gw_liquid: float, tau: Pair = (1.0, 1.0), G: float = 0.9, H: int = 40,
                         grid: Sequence[float] = (0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4, 0.5),
                         steps: int = 30000) -> Dict:
    """For an attractive liquid-only coupling (G_wA = gw_liquid < 0, G_wB = 0), the repulsive
    gas-only coupling (G_wA = 0, G_wB > 0) with the same static contact angle (meniscus
    estimator), found on a batched grid of G_wB and refined by interpolation."""
    gamma = laplace_tension(tau, G)["gamma"]
    cases = [WallCase((gw_liquid, 0.0), tuple(tau), G)] + [WallCase((0.0, g), tuple(tau), G) for g in grid]
    men = meniscus_cos(cases, gamma, H=H, steps=steps)
    target = men[0]["cos"]
    gB = match_coupling(grid, [m["cos"] for m in men[1:]], target)
    check = meniscus_cos([WallCase((0.0, gB), tuple(tau), G)], gamma, H=H, steps=steps)[0]["cos"]
    return {"gamma": gamma, "gw_liquid": gw_liquid, "cos_liquid_route": target, "gw_gas": gB,
            "cos_gas_route": check}


def _main(argv=None) -> int:
    import argparse
    import json
    ap = argparse.ArgumentParser(description="contact-angle map of the wall couplings (GPU)")
    ap.add_argument("--gw", type=float, nargs=2, action="append", metavar=("GWA", "GWB"),
                    help="a wall-coupling pair; repeat for a map")
    ap.add_argument("--tau", type=float, nargs=2, action="append", metavar=("TAUA", "TAUB"))
    ap.add_argument("--H", type=int, default=40)
    ap.add_argument("--steps", type=int, default=30000)
    a = ap.parse_args(argv)
    gws = [tuple(g) for g in (a.gw or [(-0.2, 0.2)])]
    taus = [tuple(t) for t in (a.tau or [(1.0, 1.0)])]
    m = contact_angle_map(gws, taus, H=a.H, steps=a.steps)
    for i, t in enumerate(m["taus"]):
        for j, g in enumerate(m["gws"]):
            print(json.dumps({"gw": g, "tau": t, "gamma": round(m["gammas"][t], 5),
                              "cos_meniscus": round(float(m["cos_meniscus"][i, j]), 4),
                              "cos_sessile": round(float(m["cos_sessile"][i, j]), 4),
                              "theta_meniscus_deg": round(float(m["theta_meniscus_deg"][i, j]), 2),
                              "theta_sessile_deg": round(float(m["theta_sessile_deg"][i, j]), 2),
                              "unstable": bool(m["flags"][i, j] & 2)}))
    return 0


if __name__ == "__main__":
    raise SystemExit(_main())
