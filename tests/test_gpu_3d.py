"""GPU parity of the three-dimensional (D3Q19) capillary against the FP64 3-D oracle, on the same
seeded inputs: populations after a few steps within FP32 rounding, densities within 1e-5 after
300 steps, front within 0.5 lattice units, mass within 1e-5; a z-independent slit equals the
2-D GPU channel to FP32 rounding; and a wetting duct fills.  The fused one-kernel step (the
default) equals the two-kernel step bit for bit for every row count per tile, on boxes narrower
than a tile, with ragged tiles and with the capillary touching the periodic x edge.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_0807_0602_amd import inputs
from parity_util import front_diff, max_abs_diff

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0807_0602_amd import scf
    return scf


def _fields(nx, ny, nz, liquid_x1, seed):
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    liq = X < liquid_x1
    a = np.where(liq, 2.0, 0.06) + 1e-3 * inputs.uniform_pm1(seed, 0, Y * nz + Z, X)
    b = np.where(liq, 0.06, 2.0) + 1e-3 * inputs.uniform_pm1(seed, 1, Y * nz + Z, X)
    return a, b


GEOMS = [
    ("slit", dict(nx=60, ny=12, nz=6, x0=16, x1=44, walls_y=True, walls_z=False), (-0.2, 0.2), (1.0, 1.0)),
    ("duct", dict(nx=48, ny=10, nz=10, x0=12, x1=36, walls_y=True, walls_z=True), (-0.25, 0.1), (1.2, 0.9)),
    ("open", dict(nx=33, ny=9, nz=7, x0=0, x1=0, walls_y=False, walls_z=False), (0.0, 0.0), (1.0, 0.8)),
]


def _pair(S, g, gw, tau, seed=3):
    a, b = _fields(g["nx"], g["ny"], g["nz"], max(g["x0"], g["nx"] // 3), seed)
    prm = inputs.Params(G=0.9, gw=gw, tau=tau)
    ch = S.Channel3(g["nx"], g["ny"], g["nz"], g["x0"], g["x1"], prm, a, b, walls_y=g["walls_y"],
                    walls_z=g["walls_z"])
    o = oracle.Oracle3(g["nx"], g["ny"], g["nz"], g["x0"], g["x1"], walls_y=g["walls_y"], walls_z=g["walls_z"],
                       G=0.9, gw=gw, tau=tau).init(a, b)
    return ch, o


@pytest.mark.parametrize("name,g,gw,tau", GEOMS, ids=[x[0] for x in GEOMS])
def test_populations_first_steps(S, name, g, gw, tau):
    ch, o = _pair(S, g, gw, tau)
    for steps in (0, 1, 2, 5):
        if steps:
            ch.step(steps - ch.t)
            o.step(steps - o.t)
        err = np.abs(ch.populations() - o.populations()).max()
        _say(f"  {name} step {steps}: max|df| = {err:.2e}")
        assert err <= 2e-6


@pytest.mark.parametrize("name,g,gw,tau", GEOMS[:2], ids=[x[0] for x in GEOMS[:2]])
def test_density_front_mass_300_steps(S, name, g, gw, tau):
    ch, o = _pair(S, g, gw, tau)
    worst_z = 0.0
    for t in range(0, 301, 50):
        if t:
            ch.step(50)
            o.step(50)
        a, b = ch.observe(), o.observe()
        worst_z = max(worst_z, front_diff(a["z"], b["z"]))
        for k in range(2):
            assert abs(a["mass"][k] - b["mass"][k]) / b["mass"][k] < 1e-5
        assert not a["flags"] & 2
    nA, nB = ch.density()
    rA, rB = o.density()
    err = max_abs_diff((nA, rA), (nB, rB))
    _say(f"  {name}: max|drho| = {err:.2e} max|dz| = {worst_z:.2e}")
    assert err <= 1e-5 and worst_z <= 0.5


def test_z_invariant_slit_is_the_2d_channel(S):
    case = inputs.capillary_small(seed=2)
    g, p = case.geom, case.params
    a2, b2 = case.fields()
    nz = 4
    c3 = S.Channel3(g.nx, g.ny, nz, g.x0, g.x1, p, np.repeat(a2[None], nz, 0), np.repeat(b2[None], nz, 0))
    c2 = S.Channel.from_case(case)
    c3.step(200)
    c2.step(200)
    nA3, nB3 = c3.density()
    nA2, nB2 = c2.density()
    err = max_abs_diff((nA3, np.broadcast_to(nA2[None], nA3.shape)), (nB3, np.broadcast_to(nB2[None], nB3.shape)))
    _say(f"  z-invariant slit vs 2-D channel after 200 steps: max|drho| = {err:.2e}")
    assert err <= 2e-6
    assert front_diff(c3.observe()["z"], c2.observe()["z"]) <= 1e-3


def test_wetting_duct_fills(S):
    nx, ny, nz = 160, 22, 22
    a, b = _fields(nx, ny, nz, 50, 5)
    ch = S.Channel3(nx, ny, nz, 50, 130, inputs.Params(G=0.9, gw=(-0.2, 0.2)), a, b,
                    walls_y=True, walls_z=True)
    z = []
    for _ in range(6):
        ch.step(1000)
        o = ch.observe()
        assert not o["flags"] & 2
        z.append(o["z"])
    _say(f"  duct front every 1000 steps: {np.round(z, 2).tolist()}")
    assert z[-1] > z[0] + 3.0 and np.all(np.diff(z[2:]) > 0)


SCHED_GEOMS = [
    ("duct_ragged", dict(nx=70, ny=11, nz=7, x0=9, x1=61, walls_y=True, walls_z=True), (-0.25, 0.1), (1.2, 0.9)),
    ("wall_to_edge", dict(nx=66, ny=9, nz=6, x0=0, x1=66, walls_y=True, walls_z=True), (-0.2, 0.2), (1.0, 0.8)),
    ("edge_x1", dict(nx=40, ny=8, nz=5, x0=25, x1=40, walls_y=True, walls_z=False), (0.1, -0.1), (0.9, 1.4)),
    ("edge_x0", dict(nx=40, ny=8, nz=5, x0=0, x1=17, walls_y=False, walls_z=True), (-0.3, 0.0), (1.0, 1.0)),
    ("tiny", dict(nx=3, ny=3, nz=3, x0=1, x1=2, walls_y=True, walls_z=False), (-0.2, 0.2), (1.0, 1.0)),
    ("open", dict(nx=33, ny=9, nz=7, x0=0, x1=0, walls_y=False, walls_z=False), (0.0, 0.0), (1.0, 0.8)),
]


@pytest.mark.parametrize("name,g,gw,tau", SCHED_GEOMS, ids=[x[0] for x in SCHED_GEOMS])
def test_fused_equals_two_kernel_step(S, name, g, gw, tau):
    ref, _ = _pair(S, g, gw, tau)
    ref.set_schedule(fused=False)
    assert ref.schedule()["fused"] is False
    ref.step(23)
    want = ref.populations()
    for cy in (1, 2, 5, 16, 1 << 30):
        _say(f"case: 3-D fused {name} cy={cy}, 23 steps")
        ch, _ = _pair(S, g, gw, tau)
        ch.set_schedule(fused=True, cy=cy)
        ch.step(23)
        assert np.array_equal(ch.populations(), want), cy


def test_fused_oracle_parity_on_a_ragged_duct(S):
    name, g, gw, tau = SCHED_GEOMS[0]
    ch, o = _pair(S, g, gw, tau)
    assert ch.schedule() == {"fused": True, "cy": 16}
    ch.set_schedule(fused=True, cy=4)
    ch.step(40)
    o.step(40)
    err = np.abs(ch.populations() - o.populations()).max()
    _say(f"  fused ragged duct vs oracle after 40 steps: max|df| = {err:.2e}")
    assert err <= 2e-6


def test_schedule_rejects_bad_values(S):
    from paper_0807_0602_amd import _lib as L
    name, g, gw, tau = GEOMS[1]
    ch, _ = _pair(S, g, gw, tau)
    for bad in ((2, 8), (1, 0), (-1, 4)):
        with pytest.raises(L.ScfError):
            ch.set_schedule(*bad)
    assert ch.schedule() == {"fused": True, "cy": 16}


@pytest.mark.parametrize("tau", [(1.0, 0.55), (1.0, 0.6), (1.0, 1.0)])
def test_health_flag_follows_the_oracle(S, tau):
    """The literal viscosity-ratio pairs tau_B = 0.55, 0.6 lose positivity in 3-D as in 2-D: the
    GPU's health flag (a non-finite density, or one below -1e-3 at a fluid node) is raised at the
    same steps as the same test applied to the oracle's densities; tau = (1, 1) stays clean."""
    nx, ny, nz, x0, x1 = 40, 10, 10, 10, 30
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    liq = X < 14
    a = np.where(liq, 2.0, 0.06) + 1e-3 * inputs.uniform_pm1(9, 0, Y * nz + Z, X)
    b = np.where(liq, 0.06, 2.0) + 1e-3 * inputs.uniform_pm1(9, 1, Y * nz + Z, X)
    prm = inputs.Params(G=0.9, gw=(-0.2, 0.2), tau=tau)
    ch = S.Channel3(nx, ny, nz, x0, x1, prm, a, b, walls_y=True, walls_z=True)
    o = oracle.Oracle3(nx, ny, nz, x0, x1, walls_y=True, walls_z=True, G=0.9, gw=(-0.2, 0.2), tau=tau).init(a, b)
    _say(f"case: 3-D health flag, tau={tau}")
    flags = []
    for t in range(1, 13):
        ch.step(1, allow_unstable=True)
        o.step(1)
        gpu_bad = bool(ch.observe(allow_unstable=True)["flags"] & 2)
        nA, nB = o.density()
        orc_bad = bool(not (np.isfinite(nA).all() and np.isfinite(nB).all()) or min(nA.min(), nB.min()) < -1e-3)
        flags.append((t, gpu_bad, orc_bad))
        assert gpu_bad == orc_bad, flags
    _say(f"  flags (t, gpu, oracle): {flags}")
    assert any(f[1] for f in flags) == (tau[1] < 1.0)


def test_full_size_duct_fused_equals_two_kernel(S):
    """The 3-D bench duct at its full size (512 x 182 x 182, 17.0 M nodes) in the bench's launch
    configuration (fused, 16 rows of y per tile): densities after 20 steps equal the two-kernel
    step's bit for bit; mass is conserved to FP32 rounding and no flag is raised."""
    import torch
    nx, ny, nz, x0, x1 = 512, 182, 182, 128, 384
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    liq = X < x0
    a = np.where(liq, 2.0, 0.06) + 1e-3 * inputs.uniform_pm1(1, 0, Y * nz + Z, X)
    b = np.where(liq, 0.06, 2.0) + 1e-3 * inputs.uniform_pm1(1, 1, Y * nz + Z, X)
    del Z, Y, X, liq
    prm = inputs.Params(G=0.9, gw=(-0.2, 0.2))
    _say("case: 3-D duct 512x182x182 full size, fused vs two-kernel, 20 steps")
    out = []
    for fused in (True, False):
        ch = S.Channel3(nx, ny, nz, x0, x1, prm, a, b, walls_y=True, walls_z=True)
        ch.set_schedule(fused=fused, cy=16)
        m0 = ch.observe()["mass"]
        ch.step(20)
        o = ch.observe()
        assert o["flags"] == 0
        for k in range(2):
            assert abs(o["mass"][k] - m0[k]) / m0[k] < 1e-5
        out.append(ch.density())
        del ch
        torch.cuda.empty_cache()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_largest_box_fused_equals_two_kernel(S):
    """The largest 3-D box the fused step takes: one component's 19 planes just within 4 GiB
    (512 x 332 x 332, 56.4 M nodes), where the fused kernel forms its largest unsigned 32-bit byte
    offsets (above 2^31).
    Its densities after 6 steps equal the two-kernel step's (64-bit indexing) bit for bit, with
    mass conserved and no flag."""
    import torch
    nx, ny, nz, x0, x1 = 512, 332, 332, 128, 384
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    liq = X < x0
    a = np.where(liq, 2.0, 0.06) + 1e-3 * inputs.uniform_pm1(2, 0, Y * nz + Z, X)
    b = np.where(liq, 0.06, 2.0) + 1e-3 * inputs.uniform_pm1(2, 1, Y * nz + Z, X)
    del Z, Y, X, liq
    prm = inputs.Params(G=0.9, gw=(-0.2, 0.2))
    _say("case: largest 3-D box 512x332x332, fused vs two-kernel, 6 steps")
    out = []
    for fused in (True, False):
        ch = S.Channel3(nx, ny, nz, x0, x1, prm, a, b, walls_y=True, walls_z=True)
        ch.set_schedule(fused=fused, cy=16)
        assert ch.schedule()["fused"] == fused
        m0 = ch.observe()["mass"]
        ch.step(6)
        o = ch.observe()
        assert o["flags"] == 0
        for k in range(2):
            assert abs(o["mass"][k] - m0[k]) / m0[k] < 1e-5
        out.append(ch.density())
        del ch
        torch.cuda.empty_cache()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
