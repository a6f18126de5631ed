"""Persistent schedules (SCF_ORDER_PERSIST): one block per resident slot, each walking a
contiguous run of the (channel, band, strip) tile list, the runs balanced by rows.  They change
only which block computes which node, so every persistent schedule must reproduce the default
schedule bit for bit, one or two steps per launch, with and without graphs, on edge geometries,
masks, batches of uneven channels and the full-size bench and sweep cases (with one block per CU
the sweep's blocks each run several tiles)."""
import sys

import numpy as np
import pytest

from paper_0807_0602_amd import inputs

pytestmark = pytest.mark.gpu

PERSIST, XCD = 4, 2


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


@pytest.mark.parametrize("bx", [64, 128, 256, 512])
@pytest.mark.parametrize("order", [PERSIST, PERSIST | XCD])
@pytest.mark.parametrize("fuse", [1, 2])
def test_persistent_equals_default(scf, bx, order, fuse):
    case = inputs.capillary_small(seed=2)
    _say(f"case: persistent bx={bx} order={order} fuse={fuse}, 9 and 64 steps")
    for steps, gs in ((9, 0), (64, 16)):
        a = _run(scf, case, steps, bx=256, cy=64, graph_steps=0, order=0, fuse=1)
        b = _run(scf, case, steps, bx=bx, cy=16, graph_steps=gs, order=order, fuse=fuse)
        assert b.tile()["order"] == order
        assert np.array_equal(a.populations(), b.populations()), steps


@pytest.mark.parametrize("name,geom,params", [
    ("no_walls_periodic", inputs.Geometry(70, 9, 0, 0), inputs.Params(gw=(0.0, 0.0))),
    ("fully_walled", inputs.Geometry(96, 13, 0, 96), inputs.Params(gw=(-0.2, 0.2))),
    ("odd_ny_ragged_nx", inputs.Geometry(131, 17, 20, 111), inputs.Params(gw=(-0.3, 0.3), tau=(1.5, 1.0))),
    ("tiny_box", inputs.Geometry(3, 3, 1, 2), inputs.Params(gw=(0.1, -0.1))),
    ("tall_narrow", inputs.Geometry(40, 150, 10, 30), inputs.Params(gw=(-0.25, 0.25), tau=(2.0, 0.8))),
], ids=lambda v: v if isinstance(v, str) else "")
def test_persistent_edge_geometries(scf, name, geom, params):
    case = inputs.Case(geom, params, seed=5, liquid_x1=max(geom.x0, geom.nx // 3))
    _say(f"case: persistent edge {name}, 41 steps")
    a = _run(scf, case, 41, bx=64, cy=4, graph_steps=0, fuse=1)
    for bx, fuse in ((64, 1), (64, 2), (256, 2), (512, 1)):
        b = _run(scf, case, 41, bx=bx, cy=16, graph_steps=8, order=PERSIST | XCD, fuse=fuse)
        assert np.array_equal(a.populations(), b.populations()), (bx, fuse)


def test_persistent_masked_batch(scf):
    cases = [inputs.capillary_rough(seed=1), inputs.capillary_small(seed=3),
             inputs.sweep_channel(20, 128, -0.25, 2, seed=9, steps=100, sample_every=25),
             inputs.Case(inputs.Geometry(131, 17, 20, 111), inputs.Params(gw=(-0.3, 0.3), tau=(2.0, 0.8)),
                         seed=4, liquid_x1=20)]
    _say("case: persistent batch of masked and row-walled channels, 101 steps")
    ref = scf.Batch(cases, sample_every=25, max_samples=6)
    ref.set_tile(64, 8, graph_steps=0, order=1, fuse=1)
    ref.step(101)
    for fuse in (1, 2):
        b = scf.Batch(cases, sample_every=25, max_samples=6)
        b.set_tile(256, 16, graph_steps=25, order=PERSIST | XCD, fuse=fuse)
        b.step(101)
        for i in range(len(cases)):
            ra, rb = ref.density(i)
            na, nb = b.density(i)
            assert np.array_equal(ra, na) and np.array_equal(rb, nb), (fuse, i)
        r1, n1 = ref.observe()
        r2, n2 = b.observe()
        assert n1 == n2 == 5
        for c in range(len(cases)):
            for s in range(n1):
                assert r1[c][s]["mass"] == r2[c][s]["mass"] and r1[c][s]["flags"] == r2[c][s]["flags"]


@pytest.mark.parametrize("bx", [256, 512])
def test_persistent_full_size_bitwise(scf, bx):
    """The 16384 x 1024 bench box: a persistent two-step schedule equals single steps bit for bit."""
    import torch
    case = inputs.capillary_roofline(seed=1)
    _say(f"case: persistent full size 16384x1024 bx={bx}, 4 steps")
    a = _run(scf, case, 4, bx=512, cy=8, graph_steps=0, order=1, fuse=1)
    na = a.density()
    del a
    b = _run(scf, case, 4, bx=bx, cy=16, graph_steps=0, order=PERSIST | XCD, fuse=2)
    nb = b.density()
    assert np.array_equal(na[0], nb[0]) and np.array_equal(na[1], nb[1])
    del b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("order,bpc", [(PERSIST | XCD, 0), (PERSIST, 1), (PERSIST | XCD, 1)])
def test_persistent_full_size_sweep_bitwise(scf, order, bpc):
    """The 64-channel sweep at its full size: persistent two-step schedule vs the row-band one;
    with one block per CU (256 blocks for 755 strips) every block runs several tiles."""
    import torch
    cases = inputs.sweep_draws(64, seed=0)
    _say(f"case: persistent 64-channel sweep full size, order={order} blocks_per_cu={bpc}, 6 steps")
    out = []
    for o, n in ((1, 0), (order, bpc)):
        b = scf.Batch(cases, sample_every=100, max_samples=2)
        b.set_tile(256, 8, graph_steps=0, order=o, fuse=2, blocks_per_cu=n)
        b.step(6)
        out.append([b.density(i) for i in (0, 5, 27, 40, 63)])
        del b
        torch.cuda.empty_cache()
    for (a0, a1), (b0, b1) in zip(*out):
        assert np.array_equal(a0, b0) and np.array_equal(a1, b1)
