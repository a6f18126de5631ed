"""The autotuner cache (scf_autotune_cached, scf_batch_autotune_cached): a geometry class timed
once is reused from the cache file without timing; another class, or another batch, gets its own
line; malformed lines are ignored; a cached schedule gives the same state bit for bit."""
import sys

import numpy as np
import pytest

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


def _lines(p):
    with open(p) as f:
        return [l for l in f.read().splitlines() if l.strip()]


def test_channel_cache_reuse_and_miss(scf, tmp_path):
    path = tmp_path / "tune.txt"
    path.write_text("not a cache line\n")
    case = inputs.capillary_small(seed=1)
    _say("case: autotune cache, 200 x 24 channel")
    a = scf.Channel.from_case(case)
    ta = a.autotune(3, cache=str(path))
    assert len(_lines(path)) == 2
    b = scf.Channel.from_case(case)
    tb = b.autotune(3, cache=str(path))
    assert len(_lines(path)) == 2                # reused, nothing appended
    assert {k: ta[k] for k in ("bx", "cy", "order", "fuse")} == {k: tb[k] for k in ("bx", "cy", "order", "fuse")}
    a.step(60)
    b.step(60)
    assert np.array_equal(a.populations(), b.populations())
    other = scf.Channel.from_case(inputs.Case(inputs.Geometry(128, 24, 32, 96), inputs.Params(gw=(-0.2, 0.2))))
    other.autotune(3, cache=str(path))
    assert len(_lines(path)) == 3                # another geometry class


def test_batch_cache(scf, tmp_path):
    path = str(tmp_path / "tune.txt")
    cases = [inputs.capillary_small(seed=1), inputs.sweep_channel(20, 128, -0.25, 2, seed=9, steps=100, sample_every=50)]
    _say("case: autotune cache, batch of 2")
    b1 = scf.Batch(cases, sample_every=50, max_samples=4)
    t1 = b1.autotune(2, cache=path)
    b2 = scf.Batch(cases, sample_every=50, max_samples=4)
    t2 = b2.autotune(2, cache=path)
    assert len(_lines(path)) == 1 and t1 == t2
    b3 = scf.Batch(cases[::-1], sample_every=50, max_samples=4)
    b3.autotune(2, cache=path)
    assert len(_lines(path)) == 2                # channel order is part of the class
