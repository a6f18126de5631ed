"""What the trained surrogate gains over the LBM it replaces, scored against the LBM.

Eight fresh channels are drawn like the training set (seed 5), simulated for 50 000 steps by the
batched LBM and predicted by the committed 5-input network.  The network must answer the same
curves at least 100 times faster than the LBM produced them and keep the typical per-channel
worst-case front error within a few lattice units (the exact accuracy over 64 channels is
measured and reported by bench.py --workload surrogate).  A fresh draw can fall just outside
the box of the 2000 training draws; such a channel is answered by the LBM (checked here).
"""
import os
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_0807_0602_amd", "surrogate_weights_5in.npz")


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def test_surrogate_gain_over_lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(WEIGHTS):
        pytest.skip("trained weights not present")
    from paper_0807_0602_amd import surrogate as S
    net = S.Network.load(WEIGHTS)
    cases = S.draw_cases(8, seed=5)
    _say("case: surrogate gain, 8 channels x 50000 steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    traj = S.simulate(cases, 50_000, 100)
    torch.cuda.synchronize()
    lbm_s = time.perf_counter() - t0
    errs, inside = S.curve_errors(net, cases, traj, with_length=True)
    X, _, _, _ = S.dataset(cases, traj, with_length=True)
    net.predict(X)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        net.predict(X)
    sur_s = (time.perf_counter() - t0) / 10
    ok = np.isfinite(errs[:, 0])
    _say(f"  LBM {lbm_s:.2f} s, surrogate {sur_s * 1e3:.2f} ms, speedup {lbm_s / sur_s:.0f}x, "
         f"max|dz| per channel {np.round(errs[ok, 0], 2)}, inside hull {inside:.3f}")
    assert lbm_s / sur_s > 100
    assert inside >= 0.75
    assert np.median(errs[ok, 0]) < 5.0
    # the fallback: channels with any query outside the training box come from the LBM
    t = np.arange(100, 50_001, 100, dtype=float)
    Z, P, used_lbm = S.predict_curves(net, cases, t, with_length=True)
    for c in np.nonzero(used_lbm)[0]:
        np.testing.assert_array_equal(Z[c], traj[c, 1:, 1])
