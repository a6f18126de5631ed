"""Two time steps per pass (scf_tile.fuse = 2) against single steps and the oracle.

Stage 1 of the two-step kernel computes each node with the single step's arithmetic and keeps
f*(t) on chip; stage 2 streams and collides it.  So every schedule with fuse = 2 must give the
single-step result bit for bit, for even and odd step counts (an odd remainder is one single
step), with and without graphs, for row-walled and masked channels and in batches.  The oracle
bar of the single step applies unchanged.
"""
import sys

import numpy as np
import pytest

import oracle
from parity_util import front_diff, max_abs_diff
from paper_0807_0602_amd import inputs

pytestmark = pytest.mark.gpu


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


def _run(S, case, steps, **tile):
    ch = S.Channel.from_case(case)
    if tile:
        ch.set_tile(**tile)
    ch.step(steps)
    return ch


@pytest.mark.parametrize("bx,cy,order,gs", [(64, 4, 0, 0), (128, 8, 1, 16), (256, 1 << 30, 0, 64),
                                            (512, 8, 1, 7), (64, 1, 3, 0), (256, 5, 2, 12)])
@pytest.mark.parametrize("steps", [1, 2, 9, 64])
def test_fuse2_equals_single_steps(scf, bx, cy, order, gs, steps):
    case = inputs.capillary_small(seed=2)
    _say(f"case: fuse2 bx={bx} cy={cy} order={order} graph={gs} steps={steps}")
    a = _run(scf, case, steps, bx=256, cy=64, graph_steps=0, order=0, fuse=1)
    b = _run(scf, case, steps, bx=bx, cy=cy, graph_steps=gs, order=order, fuse=2)
    assert a.t == b.t == steps
    assert np.array_equal(a.populations(), b.populations())


@pytest.mark.parametrize("name,geom,params", [
    ("no_walls_periodic", inputs.Geometry(70, 9, 0, 0), inputs.Params(gw=(0.0, 0.0))),
    ("fully_walled", inputs.Geometry(96, 13, 0, 96), inputs.Params(gw=(-0.2, 0.2))),
    ("odd_ny_ragged_nx", inputs.Geometry(131, 17, 20, 111), inputs.Params(gw=(-0.3, 0.3), tau=(1.5, 1.0))),
    ("tiny_box", inputs.Geometry(3, 3, 1, 2), inputs.Params(gw=(0.1, -0.1))),
    ("wall_to_edge", inputs.Geometry(64, 10, 32, 64), inputs.Params(gw=(-0.25, 0.25), tau=(2.0, 0.8))),
    ("general_alpha_mass", inputs.Geometry(80, 12, 20, 60),
     inputs.Params(gw=(-0.1, 0.1), alpha=(4 / 9, 0.6), mass=(1.0, 1.5), tau=(1.2, 0.9))),
], ids=lambda v: v if isinstance(v, str) else "")
def test_fuse2_edge_geometries(scf, name, geom, params):
    case = inputs.Case(geom, params, seed=5, liquid_x1=max(geom.x0, geom.nx // 3))
    _say(f"case: fuse2 edge {name}, 151 steps")
    for bx in (64, 256):
        a = _run(scf, case, 151, bx=64, cy=4, graph_steps=0, fuse=1)
        b = _run(scf, case, 151, bx=bx, cy=3, graph_steps=32, order=1, fuse=2)
        assert np.array_equal(a.populations(), b.populations()), bx
    ref = oracle.Oracle.from_case(case).init(*case.fields()).step(151).populations()
    assert np.abs(b.populations() - ref).max() <= 1e-5


def test_fuse2_masked_and_batched(scf):
    cases = [inputs.capillary_rough(seed=1), inputs.capillary_small(seed=3)]
    _say("case: fuse2 rough + row-walled batch, 121 steps")
    solo = [_run(scf, c, 121, bx=64, cy=8, graph_steps=0, fuse=1) for c in cases]
    b = scf.Batch(cases, sample_every=40, max_samples=4)
    b.set_tile(128, 6, graph_steps=40, order=1, fuse=2)
    b.step(121)
    for i, ch in enumerate(solo):
        nA, nB = ch.density()
        bA, bB = b.density(i)
        assert np.array_equal(nA, bA) and np.array_equal(nB, bB), i
    recs, n = b.observe()
    assert n == 4


def test_fuse2_parity_with_oracle(scf):
    case = inputs.capillary_small(seed=1)
    _say("case: fuse2 density and front parity, 1000 steps")
    ch = scf.Channel.from_case(case)
    ch.set_tile(256, 8, graph_steps=50, order=1, fuse=2)
    orc = oracle.Oracle.from_case(case).init(*case.fields())
    worst_z = 0.0
    for t in range(0, 1001, 100):
        if t:
            ch.step(100)
            orc.step(100)
        g, r = ch.observe(), orc.observe()
        worst_z = max(worst_z, front_diff(g["z"], r["z"]))
    nA, nB = ch.density()
    rA, rB = orc.density()
    err = max_abs_diff((nA, rA), (nB, rB))
    _say(f"  max|drho| = {err:.3e}  max|dz| = {worst_z:.3e}")
    assert err <= 1e-5 and worst_z <= 0.5


def test_fuse2_full_size_bitwise(scf):
    """The bench geometry (16384 x 1024) at the bench's schedule: two steps per pass equal two
    single steps bit for bit on the full state."""
    import torch
    case = inputs.capillary_roofline(seed=1)
    _say("case: fuse2 full size 16384x1024, 4 steps")
    a = _run(scf, case, 4, bx=512, cy=8, graph_steps=0, order=1, fuse=1)
    b = _run(scf, case, 4, bx=256, cy=16, graph_steps=0, order=3, fuse=2)
    na = a.density()
    nb = b.density()
    assert np.array_equal(na[0], nb[0]) and np.array_equal(na[1], nb[1])
    del a, b
    torch.cuda.empty_cache()


def test_fuse_rejects_bad_values(scf):
    from paper_0807_0602_amd import _lib as L
    ch = scf.Channel.from_case(inputs.capillary_small(seed=1))
    with pytest.raises(L.ScfError):
        ch.set_tile(256, 8, fuse=3)
    with pytest.raises(L.ScfError):
        ch.set_tile(256, 8, fuse=0)
    assert ch.tile()["fuse"] == 2      # the default schedule, unchanged by rejected calls
