"""GPU parity: the FP32 HIP path against the FP64 CPU oracle on the same seeded inputs.

Bar (FP32 state vs FP64 oracle): max |n_k^GPU - n_k^oracle| <= 1e-5 after 1000 steps of the
200 x 24 capillary, |z^GPU - z^oracle| <= 0.5 lattice units through 2000 steps.  Variants of
the GPU path (tile shapes, graph or eager launches, fused or two-kernel, batched or solo,
checkpoint round trip) must agree bit for bit: they run identical per-node arithmetic.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_0807_0602_amd import inputs
from parity_util import front_diff, max_abs_diff

pytestmark = pytest.mark.gpu

RHO_TOL = 1e-5
Z_TOL = 0.5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def scf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0807_0602_amd import scf as S
    return S


def _oracle_run(case, steps):
    return oracle.Oracle.from_case(case).init(*case.fields()).step(steps)


# ------------------------------------------------------------------------------ populations
@pytest.mark.parametrize("steps", [0, 1, 2, 7])
def test_populations_first_steps(scf, steps):
    case = inputs.capillary_small(seed=1)
    _say(f"case: populations {case.name} steps={steps}")
    ch = scf.Channel.from_case(case)
    ch.step(steps)
    f = ch.populations()
    ref = _oracle_run(case, steps).populations()
    np.testing.assert_allclose(f, ref, rtol=0, atol=2e-6)


# ------------------------------------------------------------------------------ densities
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_density_parity_1000_steps(scf, seed):
    case = inputs.capillary_small(seed=seed)
    _say(f"case: density parity {case.name} seed={seed} 1000 steps")
    ch = scf.Channel.from_case(case)
    ch.step(1000)
    nA, nB = ch.density()
    rA, rB = _oracle_run(case, 1000).density()
    err = max_abs_diff((nA, rA), (nB, rB))
    _say(f"  max|drho| = {err:.3e}")
    assert err <= RHO_TOL


def test_front_and_mass_through_2000_steps(scf):
    case = inputs.capillary_small(seed=1)
    _say(f"case: z(t) parity {case.name} 2000 steps, every 10")
    ch = scf.Channel.from_case(case)
    orc = oracle.Oracle.from_case(case).init(*case.fields())
    m0 = ch.observe()["mass"]
    worst_z = worst_p = 0.0
    for t in range(0, 2001, 10):
        if t:
            ch.step(10)
            orc.step(10)
        g, r = ch.observe(), orc.observe()
        assert g["t"] == r["t"] == t
        worst_z = max(worst_z, front_diff(g["z"], r["z"]))
        worst_p = max(worst_p, front_diff(g["precursor"], r["precursor"]))
        assert g["flags"] == r["flags"]
        for k in range(2):
            assert abs(g["mass"][k] - r["mass"][k]) / r["mass"][k] < 1e-5
    _say(f"  max|dz| = {worst_z:.3e}  max|dp| = {worst_p:.3e}")
    assert worst_z <= Z_TOL
    assert worst_p <= Z_TOL
    m1 = ch.observe()["mass"]
    for k in range(2):
        assert abs(m1[k] - m0[k]) / m0[k] < 1e-5     # FP32 drift stays small


# ------------------------------------------------------------------------------ edge geometries
EDGE_CASES = [
    # (name, geometry, params, fields builder)
    ("no_walls_periodic", inputs.Geometry(70, 9, 0, 0), inputs.Params(gw=(0.0, 0.0))),
    ("fully_walled", inputs.Geometry(96, 13, 0, 96), inputs.Params(gw=(-0.2, 0.2))),
    ("odd_ny_ragged_nx", inputs.Geometry(131, 17, 20, 111), inputs.Params(gw=(-0.3, 0.3), tau=(1.5, 1.0))),
    ("tiny_box", inputs.Geometry(3, 3, 1, 2), inputs.Params(gw=(0.1, -0.1))),
    ("wall_to_edge", inputs.Geometry(64, 10, 32, 64), inputs.Params(gw=(-0.25, 0.25), tau=(2.0, 0.8))),
    ("general_alpha_mass", inputs.Geometry(80, 12, 20, 60),
     inputs.Params(gw=(-0.1, 0.1), alpha=(4 / 9, 0.6), mass=(1.0, 1.5), tau=(1.2, 0.9))),
]


@pytest.mark.parametrize("name,geom,params", EDGE_CASES, ids=[c[0] for c in EDGE_CASES])
def test_edge_geometries(scf, name, geom, params):
    case = inputs.Case(geom, params, seed=5, liquid_x1=max(geom.x0, geom.nx // 3))
    steps = 150
    _say(f"case: edge {name} {geom} {steps} steps")
    ch = scf.Channel.from_case(case)
    ch.step(steps)
    f = ch.populations()
    ref = _oracle_run(case, steps).populations()
    err = np.abs(f - ref).max()
    _say(f"  max|df| = {err:.3e}")
    assert err <= 1e-5


# ------------------------------------------------------------------------------ bitwise variants
def _state(ch):
    return ch.populations()


@pytest.mark.parametrize("bx,cy,order", [(64, 8, 0), (64, 1 << 30, 0), (128, 5, 0), (256, 64, 0),
                                         (256, 1, 0), (128, 23, 0), (64, 4, 1), (256, 7, 1), (128, 1, 1),
                                         (64, 3, 2), (256, 16, 3), (128, 1, 3), (512, 8, 1), (512, 1 << 30, 2)])
def test_tile_shapes_bitwise(scf, bx, cy, order):
    case = inputs.capillary_small(seed=2)
    _say(f"case: tile shape bx={bx} cy={cy} order={order}")
    a = scf.Channel.from_case(case)
    a.step(120)
    b = scf.Channel.from_case(case)
    b.set_tile(bx, cy, 64, order)
    b.step(120)
    assert np.array_equal(_state(a), _state(b))


def test_graph_vs_eager_bitwise(scf):
    case = inputs.capillary_small(seed=3)
    _say("case: graph vs eager")
    a = scf.Channel.from_case(case)
    a.set_tile(256, 64, 0)
    a.step(257)
    b = scf.Channel.from_case(case)
    b.set_tile(256, 64, 32)
    for _ in range(3):       # replay the captured graphs several times, eager tail in between
        b.step(85)
    b.step(2)
    assert a.t == b.t == 257
    assert np.array_equal(_state(a), _state(b))


def test_two_kernel_matches_fused_bitwise(scf):
    case = inputs.capillary_small(seed=1)
    _say("case: two-kernel vs fused")
    from paper_0807_0602_amd import _lib as L
    a = scf.Channel.from_case(case)
    a.step(300)
    b = scf.Channel.from_case(case)
    b.set_variant(L.SCF_VARIANT_TWO_KERNEL)
    b.step(300)
    assert np.array_equal(_state(a), _state(b))


def test_checkpoint_roundtrip_bitwise(scf, tmp_path):
    case = inputs.capillary_small(seed=1)
    _say("case: checkpoint round trip")
    a = scf.Channel.from_case(case)
    a.step(400)
    b = scf.Channel.from_case(case)
    b.step(200)
    p = str(tmp_path / "ck.bin")
    b.save(p)
    c = scf.Channel.from_case(case)
    c.load(p)
    assert c.t == 200
    c.step(200)
    assert np.array_equal(_state(a), _state(c))


def test_checkpoint_rejects_other_geometry(scf, tmp_path):
    from paper_0807_0602_amd import _lib as L
    a = scf.Channel.from_case(inputs.capillary_small(seed=1))
    p = str(tmp_path / "ck.bin")
    a.save(p)
    other = inputs.Case(inputs.Geometry(128, 24, 32, 96), inputs.Params(gw=(-0.2, 0.2)))
    b = scf.Channel.from_case(other)
    with pytest.raises(L.ScfError) as e:
        b.load(p)
    assert e.value.code == L.SCF_ESTATE


# ------------------------------------------------------------------------------ errors, instability
def test_rejects_tau_at_one_half(scf):
    from paper_0807_0602_amd import _lib as L
    case = inputs.with_params(inputs.capillary_small(), tau=(1.0, 0.5))
    with pytest.raises(L.ScfError) as e:
        scf.Channel.from_case(case)
    assert e.value.code == L.SCF_EINVAL


def test_instability_is_flagged(scf):
    """tau_B = 0.55 with tau_A = 1 goes unstable on the 200 x 24 capillary: both the oracle and
    the GPU must report it (health flag bit 1, SCF_EUNSTABLE), and after that observation the
    next scf_step reports it too (lazily, after enqueueing its steps)."""
    from paper_0807_0602_amd import _lib as L
    case = inputs.with_params(inputs.capillary_small(seed=1), tau=(1.0, 0.55))
    _say("case: instability flag, tau = (1.0, 0.55)")
    orc = oracle.Oracle.from_case(case).init(*case.fields())
    ch = scf.Channel.from_case(case)
    t_orc = t_gpu = None
    for t in range(100, 3001, 100):
        orc.step(100)
        if t_gpu is None:
            ch.step(100)                  # no observation has found instability yet
        else:
            with pytest.raises(L.ScfError) as e:
                ch.step(100)
            assert e.value.code == L.SCF_EUNSTABLE
        if t_orc is None and orc.observe()["flags"] & 2:
            t_orc = t
        if t_gpu is None:
            o = ch.observe(allow_unstable=True)
            if o["flags"] & 2:
                t_gpu = t
                with pytest.raises(L.ScfError) as e:
                    ch.observe()
                assert e.value.code == L.SCF_EUNSTABLE
        if t_orc and t_gpu:
            break
    _say(f"  flagged at oracle t={t_orc}, gpu t={t_gpu}")
    assert t_orc is not None and t_gpu is not None


# ------------------------------------------------------------------------------ batched
def test_batch_matches_solo_bitwise(scf):
    cases = [inputs.capillary_small(seed=1),
             inputs.sweep_channel(20, 128, -0.25, 2, seed=9, steps=300, sample_every=50),
             inputs.Case(inputs.Geometry(131, 17, 20, 111), inputs.Params(gw=(-0.3, 0.3), tau=(2.0, 0.8)),
                         seed=4, liquid_x1=20)]
    _say("case: batch of 3 vs solo")
    b = scf.Batch(cases, sample_every=50, max_samples=8)
    b.step(300)
    recs, ns = b.observe()
    assert ns == 7
    for c, case in enumerate(cases):
        solo = scf.Channel.from_case(case)
        for s in range(7):
            o = solo.observe()
            r = recs[c][s]
            assert r["t"] == s * 50 == o["t"]
            for key in ("z", "precursor", "precursor_lo", "precursor_hi"):
                assert (math.isnan(r[key]) and math.isnan(o[key])) or r[key] == o[key], (c, s, key)
            assert r["mass"] == o["mass"] and r["flags"] == o["flags"]
            if s < 6:
                solo.step(50)
        da = b.density(c)
        ds = solo.density()
        assert np.array_equal(da[0], ds[0]) and np.array_equal(da[1], ds[1])


def test_batch_against_oracle(scf):
    cases = [inputs.sweep_channel(20, 128, g, r, seed=10 + i, steps=500, sample_every=100)
             for i, (g, r) in enumerate([(-0.3, 1), (0.2, 2), (-0.1, 5), (-0.25, 10)])]
    _say("case: batch of 4 sweep channels vs oracle, 500 steps")
    b = scf.Batch(cases, sample_every=100, max_samples=6)
    b.autotune(3)
    b.step(500)
    recs, ns = b.observe()
    assert ns == 6
    for c, case in enumerate(cases):
        orc = oracle.Oracle.from_case(case).init(*case.fields())
        for s in range(ns):
            r, o = recs[c][s], orc.observe()
            assert front_diff(r["z"], o["z"]) <= Z_TOL
            orc.step(100)
        nA, nB = b.density(c)
        orc2 = oracle.Oracle.from_case(case).init(*case.fields()).step(500)
        rA, rB = orc2.density()
        assert max_abs_diff((nA, rA), (nB, rB)) <= RHO_TOL


# ------------------------------------------------------------------------------ full sizes
# the schedule bench.py's autotuner picks for the 16384 x 1024 capillary (two steps per launch,
# 256-wide blocks on 224-column strips, persistent strip-aligned bands in XCD eighths)
BENCH_TILE = dict(bx=256, cy=16, graph_steps=64, order=6, fuse=2)


def _window_check(scf, case, T, centres, half, tile=BENCH_TILE):
    """Run the full-size GPU channel T steps in the bench's launch configuration; for each sampled
    centre column, run the oracle on a window of width 2*half+1 (x clamped at its edges) and
    compare the columns at distance > 2T from the window edges, where the window's result is
    exact."""
    ch = scf.Channel.from_case(case)
    ch.set_tile(**tile)
    ch.step(T)
    nA, nB = ch.density()
    return _windows_of(case, nA, nB, T, centres, half)


def _windows_of(case, nA, nB, T, centres, half):
    """Largest density difference between the GPU fields (nA, nB after T steps) and the oracle
    run on windows around the given columns (see _window_check)."""
    assert np.isfinite(nA).all() and np.isfinite(nB).all(), "non-finite GPU density"
    worst = 0.0
    nx = case.geom.nx
    for xc in centres:
        xa = xc - half
        w = 2 * half + 1
        orc = oracle.Oracle.from_case(case, periodic_x=False, x_offset=xa, width=w)
        orc.init(*case.fields(xa, xa + w)).step(T)
        rA, rB = orc.density()
        inner = np.arange(2 * T + 1, w - 2 * T - 1)
        cols = (xa + inner) % nx
        worst = max(worst, max_abs_diff((nA[:, cols], rA[:, inner]), (nB[:, cols], rB[:, inner])))
    return worst


def test_full_size_roofline_case_windows(scf):
    case = inputs.capillary_roofline(seed=1)
    T = 60
    _say(f"case: {case.name} full size, {T} steps, oracle windows")
    g = case.geom
    # channel inlet, channel outlet, the x = 0 wrap, a bulk column
    worst = _window_check(scf, case, T, [g.x0, g.x1 - 1, 0, 7000], half=2 * T + 8)
    _say(f"  max|drho| = {worst:.3e}")
    assert worst <= RHO_TOL


def test_full_size_washburn_case_windows(scf):
    case = inputs.capillary_washburn(seed=1)
    T = 100
    _say(f"case: {case.name} full size, {T} steps, oracle windows")
    g = case.geom
    # the schedule the autotuner picks for this size (bench.py --workload washburn)
    worst = _window_check(scf, case, T, [g.x0, g.x1, 4095], half=2 * T + 6,
                          tile=dict(bx=64, cy=8, graph_steps=64, order=3, fuse=2))
    _say(f"  max|drho| = {worst:.3e}")
    assert worst <= RHO_TOL


def test_full_size_sweep_batch_windows(scf):
    """The 64-channel calibration sweep at its full size (12.9 M nodes, one launch per two steps
    for all channels) in the schedule the sweep bench's autotuner picks; oracle windows on the
    longest and the shortest channel and on channel 27 (the one that loses stability late)."""
    import torch
    cases = inputs.sweep_draws(64, seed=0)
    T = 50
    _say(f"case: 64-channel sweep full size, {T} steps, oracle windows on three channels")
    b = scf.Batch(cases, sample_every=100, max_samples=2)
    b.set_tile(256, 8, graph_steps=100, order=1, fuse=2)
    b.step(T)
    nxs = [c.geom.nx for c in cases]
    picks = sorted({int(np.argmax(nxs)), int(np.argmin(nxs)), 27})
    worst = 0.0
    for i in picks:
        c = cases[i]
        nA, nB = b.density(i)
        g = c.geom
        worst = max(worst, _windows_of(c, nA, nB, T, [g.x0, g.x1 - 1, 0], half=2 * T + 8))
    _say(f"  channels {picks}: max|drho| = {worst:.3e}")
    assert worst <= RHO_TOL
    del b
    torch.cuda.empty_cache()


def test_full_size_roofline_case_mass_and_observables(scf):
    """Properties that hold at any size: mass conservation and the initial front z(0) = -1/2."""
    case = inputs.capillary_roofline(seed=2)
    _say(f"case: {case.name} mass over 200 steps")
    ch = scf.Channel.from_case(case)
    ch.set_tile(**BENCH_TILE)
    o0 = ch.observe()
    assert abs(o0["z"] + 0.5) < 0.01
    ch.step(200)
    o1 = ch.observe()
    for k in range(2):
        assert abs(o1["mass"][k] - o0["mass"][k]) / o0["mass"][k] < 1e-5
    assert o1["flags"] == 0


def test_largest_channel_bitwise(scf):
    """The largest channel one context takes: one population buffer just within 4 GiB (16384 x
    3640, 59.6 M nodes), where the fused kernels form their largest unsigned 32-bit byte offsets
    (above 2^31).  The default two-step schedule and the two-kernel step (64-bit indexing) give
    the same densities bit for bit after 6 steps, with mass conserved and no flag."""
    import torch
    from paper_0807_0602_amd import _lib as L
    geom = inputs.Geometry(16384, 3640, 4096, 12288)
    case = inputs.Case(geom, inputs.Params(G=0.9, gw=(-0.2, 0.2)), seed=4, liquid_x1=4096)
    _say("case: largest channel 16384x3640, two-step default vs two-kernel, 6 steps")
    out = []
    for two_kernel in (False, True):
        ch = scf.Channel.from_case(case)
        if two_kernel:
            ch.set_variant(L.SCF_VARIANT_TWO_KERNEL)
        else:
            ch.set_tile(**BENCH_TILE)
        m0 = ch.observe()["mass"]
        ch.step(6)
        o = ch.observe()
        assert o["flags"] == 0
        for k in range(2):
            assert abs(o["mass"][k] - m0[k]) / m0[k] < 1e-5
        out.append(ch.density())
        ch.close()
        del ch
        torch.cuda.empty_cache()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
