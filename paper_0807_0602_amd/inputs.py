"""Seeded synthetic inputs for the binary Shan-Chen capillary-filling model.

This module only builds input fields and parameter sets.  It holds none of the
model's arithmetic (no equilibrium, force, collision or streaming), so both the
FP64 CPU oracle and the HIP library can be fed from it without sharing any of
the method's code.

Geometry convention (Sec. 3 of the paper, Fig. 1): a box of nx by ny nodes,
periodic in x and y.  Rows y = 0 and y = ny-1 are solid for x in [x0, x1): that
is the coated capillary.  Outside [x0, x1) those rows are fluid and periodic in
y, which is the "infinite reservoir".  With half-way bounce-back the channel
height is H = ny - 2 fluid rows.  The incoming liquid (component A) fills
x < x0 at t = 0, the displaced fluid (component B) fills x >= x0.

Noise: an additive uniform perturbation in [-amp, amp) per component and fluid
node, from SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) applied to a counter built from
(seed, component, y, x).  Because the counter holds the global node position,
any window of a field can be regenerated exactly on its own.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Sequence, Tuple

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function of a uint64 counter array (published constants)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, comp: int, ys: np.ndarray, xs: np.ndarray) -> np.ndarray:
    """Uniform values in [-1, 1) for every (y, x) pair of the broadcast grids ys, xs.

    The counter is seed*2^48 + comp*2^40 + y*2^20 + x, so x and y must stay below 2^20.
    """
    ys = np.asarray(ys, dtype=np.uint64)
    xs = np.asarray(xs, dtype=np.uint64)
    base = (np.uint64(seed) << np.uint64(48)) | (np.uint64(comp) << np.uint64(40))
    ctr = base | (ys << np.uint64(20)) | xs
    h = splitmix64(ctr)
    u = (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)  # 53-bit in [0,1)
    return 2.0 * u - 1.0


@dataclass(frozen=True)
class Geometry:
    """Box nx by ny, periodic in x and y, solid rows y=0 and y=ny-1 over x in [x0, x1).

    ``solid`` (optional, (ny, nx), non-zero = solid) replaces the rows as the set of solid
    nodes; x0 and x1 then only place the observables (inlet x0, reservoir centre x0/2).
    """
    nx: int
    ny: int
    x0: int = 0
    x1: int = 0
    solid: Optional[np.ndarray] = field(default=None, compare=False, repr=False)

    def solid_mask(self) -> np.ndarray:
        if self.solid is not None:
            m = np.asarray(self.solid) != 0
            assert m.shape == (self.ny, self.nx)
            return m.copy()
        m = np.zeros((self.ny, self.nx), dtype=bool)
        if self.x1 > self.x0:
            m[0, self.x0:self.x1] = True
            m[self.ny - 1, self.x0:self.x1] = True
        return m

    @property
    def H(self) -> int:
        return self.ny - 2


@dataclass(frozen=True)
class Params:
    """Model parameters in lattice units.

    G       inter-component coupling; the neighbour weights are 1/9 (axis) and 1/36 (diagonal)
    gw      wall couplings (G_wA, G_wB) with the wall density folded in; negative attracts
    tau     relaxation times (tau_A, tau_B), each > 1/2
    alpha   rest fractions of the equilibrium (4/9 gives the usual D2Q9 weights)
    mass    molecular masses m_k (rho_k = m_k n_k)
    """
    G: float = 0.9
    gw: Tuple[float, float] = (0.0, 0.0)
    tau: Tuple[float, float] = (1.0, 1.0)
    alpha: Tuple[float, float] = (4.0 / 9.0, 4.0 / 9.0)
    mass: Tuple[float, float] = (1.0, 1.0)


@dataclass(frozen=True)
class Case:
    """A complete seeded problem: geometry, parameters and the initial density recipe."""
    geom: Geometry
    params: Params
    rho_liq: float = 2.0      # majority density of each component in its own phase
    rho_min: float = 0.06     # minority (dissolved) density
    gas: Optional[Tuple[float, float]] = None   # (n_A, n_B) of the B-rich phase if not symmetric
    liquid_x1: Optional[int] = None   # liquid A fills x < liquid_x1 (default x0)
    noise: float = 1e-3
    seed: int = 1
    steps: int = 2000
    sample_every: int = 10
    name: str = ""

    def fields(self, xa: int = 0, xb: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
        """Initial (rhoA, rhoB), shape (ny, xb-xa), for global columns xa..xb-1 (taken mod nx)."""
        g = self.geom
        if xb is None:
            xb = xa + g.nx
        xs_glob = np.arange(xa, xb) % g.nx
        ys = np.arange(g.ny)
        Y, X = np.meshgrid(ys, xs_glob, indexing="ij")
        lx1 = g.x0 if self.liquid_x1 is None else self.liquid_x1
        liquid = X < lx1
        gA, gB = self.gas if self.gas is not None else (self.rho_min, self.rho_liq)
        rhoA = np.where(liquid, self.rho_liq, gA).astype(np.float64)
        rhoB = np.where(liquid, self.rho_min, gB).astype(np.float64)
        if self.noise:
            rhoA = rhoA + self.noise * uniform_pm1(self.seed, 0, Y, X)
            rhoB = rhoB + self.noise * uniform_pm1(self.seed, 1, Y, X)
        solid = g.solid_mask()[:, xs_glob]
        rhoA[solid] = 0.0
        rhoB[solid] = 0.0
        return np.ascontiguousarray(rhoA), np.ascontiguousarray(rhoB)


# ---------------------------------------------------------------------------------------------
# The workloads of the build.  Each is a channel of height H = ny-2 between a liquid reservoir
# (x < x0) and a gas reservoir (x >= x1); x wraps, so the two reservoirs touch at x = 0.
# ---------------------------------------------------------------------------------------------

def capillary_small(seed: int = 1) -> Case:
    """200 x 24 box, channel x in [50,150), H = 22, G_w = (-0.2, +0.2), tau = (1, 1)."""
    return Case(Geometry(200, 24, 50, 150), Params(G=0.9, gw=(-0.2, 0.2), tau=(1.0, 1.0)),
                seed=seed, steps=2000, sample_every=10, name="capillary_200x24")


def rough_mask(nx: int, ny: int, x0: int, x1: int, seed: int, bumps: int = 12,
               post: Optional[Tuple[int, int, int, int]] = None) -> np.ndarray:
    """Solid mask of a capillary with rough walls: the wall rows over [x0, x1) plus `bumps`
    one- or two-node-high steps on each wall at seeded positions, and an optional solid post
    (xa, xb, ya, yb) inside the channel.  Geometry only; no model arithmetic."""
    m = np.zeros((ny, nx), dtype=np.uint8)
    m[0, x0:x1] = 1
    m[ny - 1, x0:x1] = 1
    rng = np.random.default_rng(seed)
    for wall in (0, 1):
        xs = rng.integers(x0, max(x0 + 1, x1 - 3), size=bumps)
        ws = rng.integers(1, 4, size=bumps)
        hs = rng.integers(1, 3, size=bumps)
        for x, w, h in zip(xs, ws, hs):
            rows = range(1, 1 + h) if wall == 0 else range(ny - 1 - h, ny - 1)
            for y in rows:
                m[y, x:min(x + w, x1)] = 1
    if post is not None:
        xa, xb, ya, yb = post
        m[ya:yb, xa:xb] = 1
    return m


def capillary_rough(seed: int = 1, post: bool = True) -> Case:
    """The 200 x 24 capillary with rough walls (seeded steps on both walls) and, optionally, a
    4 x 4 solid post at x = 96..100, y = 6..9, below the centre line (general solid mask)."""
    nx, ny, x0, x1 = 200, 24, 50, 150
    m = rough_mask(nx, ny, x0, x1, seed=100 + seed, post=(96, 100, 6, 10) if post else None)
    return Case(Geometry(nx, ny, x0, x1, solid=m), Params(G=0.9, gw=(-0.2, 0.2), tau=(1.0, 1.0)),
                seed=seed, steps=2000, sample_every=10, name="capillary_rough_200x24")


# Relaxation-time pairs (tau_A, tau_B) realising a dynamic-viscosity ratio r = nu_A/nu_B between
# the liquid phase (mostly A) and the gas phase (mostly B), whose densities are both about 2.0.
# The pairs with tau_A = 1 and tau_B = 0.5 + 0.5/r lose positivity for r >= 2 under plain BGK at
# G = 0.9, so the working pairs keep both tau well above 1/2.  Literal pairs stay available to
# exercise the instability flag.
TAU_FOR_RATIO = {1: (1.0, 1.0), 2: (1.5, 1.0), 5: (2.0, 0.8), 10: (3.0, 0.75)}
TAU_LITERAL_FOR_RATIO = {r: (1.0, 0.5 + 0.5 / r) for r in (1, 2, 5, 10)}


def capillary_washburn(tau: Tuple[float, float] = TAU_FOR_RATIO[10], seed: int = 1) -> Case:
    """4096 x 202 box, channel x in [512, 3584), H = 200, G_w = (-0.25, +0.25)."""
    return Case(Geometry(4096, 202, 512, 3584), Params(G=0.9, gw=(-0.25, 0.25), tau=tau),
                seed=seed, steps=200_000, sample_every=100, name="capillary_4096x202")


def capillary_roofline(seed: int = 1) -> Case:
    """16384 x 1024 box, walls over the central half x in [4096, 12288), tau = (1, 1)."""
    return Case(Geometry(16384, 1024, 4096, 12288), Params(G=0.9, gw=(-0.2, 0.2), tau=(1.0, 1.0)),
                seed=seed, steps=10_000, sample_every=100, name="capillary_16384x1024")


def sweep_channel(H: int, L: int, gwA: float, ratio: int, seed: int, literal_tau: bool = False,
                  steps: int = 50_000, sample_every: int = 100) -> Case:
    """One channel of the calibration sweep: nx = 1.5 L, ny = H + 2, channel x in [L/4, 5L/4)."""
    tau = (TAU_LITERAL_FOR_RATIO if literal_tau else TAU_FOR_RATIO)[ratio]
    nx = (3 * L) // 2
    geom = Geometry(nx, H + 2, L // 4, (5 * L) // 4)
    return Case(geom, Params(G=0.9, gw=(gwA, -gwA), tau=tau), seed=seed, steps=steps,
                sample_every=sample_every, name=f"sweep_H{H}_L{L}_r{ratio}")


def sweep_draws(n: int = 64, seed: int = 0, H_set: Sequence[int] = (20, 40, 80, 160),
                L_set: Sequence[int] = (512, 1024, 2048, 4096), ratios: Sequence[int] = (1, 2, 5, 10),
                gw_range: Tuple[float, float] = (-0.3, 0.3), steps: int = 50_000,
                sample_every: int = 100) -> list:
    """n channels with H, L and r uniform over their sets and G_wA uniform in gw_range."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n):
        H = int(rng.choice(H_set))
        L = int(rng.choice(L_set))
        r = int(rng.choice(ratios))
        gwA = float(rng.uniform(*gw_range))
        out.append(sweep_channel(H, L, gwA, r, seed=1000 * (seed + 1) + c, steps=steps,
                                 sample_every=sample_every))
    return out


def flat_slab(nx: int = 128, ny: int = 4, tau=(1.0, 1.0), seed: int = 0, noise: float = 0.0) -> Case:
    """Periodic box with no walls; liquid A in the middle half of x, B elsewhere."""
    return Case(Geometry(nx, ny, 0, 0), Params(G=0.9, gw=(0.0, 0.0), tau=tau),
                liquid_x1=None, noise=noise, seed=seed, name=f"slab_{nx}x{ny}")


def slab_fields(case: Case) -> Tuple[np.ndarray, np.ndarray]:
    """Liquid A for x in [nx/4, 3nx/4), B elsewhere (two flat interfaces)."""
    g = case.geom
    X = np.broadcast_to(np.arange(g.nx)[None, :], (g.ny, g.nx))
    Y = np.broadcast_to(np.arange(g.ny)[:, None], (g.ny, g.nx))
    liquid = (X >= g.nx // 4) & (X < 3 * g.nx // 4)
    rhoA = np.where(liquid, case.rho_liq, case.rho_min).astype(np.float64)
    rhoB = np.where(liquid, case.rho_min, case.rho_liq).astype(np.float64)
    if case.noise:
        rhoA = rhoA + case.noise * uniform_pm1(case.seed, 0, Y, X)
        rhoB = rhoB + case.noise * uniform_pm1(case.seed, 1, Y, X)
    return np.ascontiguousarray(rhoA), np.ascontiguousarray(rhoB)


def droplet_fields(n: int, R: float, rho_liq: float = 2.0, rho_min: float = 0.06,
                   noise: float = 0.0, seed: int = 0,
                   gas: Optional[Tuple[float, float]] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Periodic n x n box, a disc of A of radius R centred at ((n-1)/2, (n-1)/2) in B.
    `gas`: (n_A, n_B) outside the disc, default (rho_min, rho_liq)."""
    c = (n - 1) / 2.0
    Y, X = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    inside = (X - c) ** 2 + (Y - c) ** 2 < R * R
    gA, gB = gas if gas is not None else (rho_min, rho_liq)
    rhoA = np.where(inside, rho_liq, gA).astype(np.float64)
    rhoB = np.where(inside, rho_min, gB).astype(np.float64)
    if noise:
        rhoA = rhoA + noise * uniform_pm1(seed, 0, Y, X)
        rhoB = rhoB + noise * uniform_pm1(seed, 1, Y, X)
    return np.ascontiguousarray(rhoA), np.ascontiguousarray(rhoB)


def plug_fields(geom: Geometry, xa: int, xb: int, rho_liq: float = 2.0,
                rho_min: float = 0.06, gas: Optional[Tuple[float, float]] = None) -> Tuple[np.ndarray, np.ndarray]:
    """A plug of A for x in [xa, xb) in a channel; B elsewhere (composition `gas`, default
    (rho_min, rho_liq)); solid nodes zero."""
    Y, X = np.meshgrid(np.arange(geom.ny), np.arange(geom.nx), indexing="ij")
    inside = (X >= xa) & (X < xb)
    gA, gB = gas if gas is not None else (rho_min, rho_liq)
    rhoA = np.where(inside, rho_liq, gA).astype(np.float64)
    rhoB = np.where(inside, rho_min, gB).astype(np.float64)
    solid = geom.solid_mask()
    rhoA[solid] = 0.0
    rhoB[solid] = 0.0
    return np.ascontiguousarray(rhoA), np.ascontiguousarray(rhoB)


def sessile_fields(geom: Geometry, xc: float, R: float, rho_liq: float = 2.0,
                   rho_min: float = 0.06, gas: Optional[Tuple[float, float]] = None) -> Tuple[np.ndarray, np.ndarray]:
    """A half-disc of A of radius R centred at (xc, 0.5) on the bottom wall plane (between the
    solid row 0 and the first fluid row), B elsewhere (composition `gas`, default
    (rho_min, rho_liq)); solid nodes zero."""
    Y, X = np.meshgrid(np.arange(geom.ny), np.arange(geom.nx), indexing="ij")
    inside = (X - xc) ** 2 + (Y - 0.5) ** 2 < R * R
    gA, gB = gas if gas is not None else (rho_min, rho_liq)
    rhoA = np.where(inside, rho_liq, gA).astype(np.float64)
    rhoB = np.where(inside, rho_min, gB).astype(np.float64)
    solid = geom.solid_mask()
    rhoA[solid] = 0.0
    rhoB[solid] = 0.0
    return np.ascontiguousarray(rhoA), np.ascontiguousarray(rhoB)


def with_params(case: Case, **kw) -> Case:
    """Copy of a case with some Params fields replaced."""
    return replace(case, params=replace(case.params, **kw))
