"""A sweep channel that loses stability: channel 27 of the 64-channel calibration sweep (H = 20,
L = 512, tau = (1.5, 1.0), G_wA = -0.237) fills steadily and then develops a non-finite density
at step 17 100 in the FP64 oracle (tests/golden/sweep_instability_H20_L512_r2.json, written by
tests/golden/make_sweep_instability.py, which runs only the oracle).  The FP32 GPU run must track
the oracle's front every 1000 steps to 0.5 lattice units and raise the health flag within 300
steps of the oracle's first unstable observation: the flag is the model's, not the precision's.
"""
import json
import os
import sys

import pytest

from paper_0807_0602_amd import inputs
from parity_util import front_diff

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sweep_instability_H20_L512_r2.json")


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


@pytest.mark.parametrize("fuse", [1, 2])
def test_sweep_channel_goes_unstable_with_the_oracle(scf, fuse):
    ref = json.load(open(GOLDEN))
    case = inputs.sweep_draws(64, seed=0)[ref["case"]["index"]]
    _say(f"case: {case.name} fuse={fuse}, until the health flag (oracle: t = {ref['first_unstable_t']})")
    ch = scf.Channel.from_case(case)
    ch.set_tile(256, 16, graph_steps=0, order=0, fuse=fuse)
    first_bad = None
    worst = 0.0
    for t in range(100, ref["first_unstable_t"] + 1001, 100):
        ch.step(100)
        o = ch.observe(allow_unstable=True)
        if o["flags"] & 2:
            first_bad = t
            break
        if str(t) in ref["z_every_1000"]:
            worst = max(worst, front_diff(o["z"], ref["z_every_1000"][str(t)]))
    _say(f"  GPU first unstable t = {first_bad}, max|dz| before = {worst:.3e}")
    assert worst <= 0.5
    assert first_bad is not None and abs(first_bad - ref["first_unstable_t"]) <= 300
