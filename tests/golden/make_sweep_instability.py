"""Writes sweep_instability_H20_L512_r2.json with the FP64 oracle (run from the repository root:
python tests/golden/make_sweep_instability.py).

Channel 27 of the 64-channel calibration sweep (draw seed 0): H = 20, L = 512, viscosity ratio 2
realised as tau = (1.5, 1.0), G_wA = -0.2367.  The oracle advances it in blocks of 100 steps and
records the front z on the centre line every 1000 steps and the first observation
at which the health flag reports a non-finite or negative density.  The state of eq. lbe at
these parameters loses positivity late in the filling, so the flag is a property of the model,
which the GPU run must reproduce.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_0807_0602_amd import inputs  # noqa: E402

INDEX = 27
LIMIT = 20_000


def main() -> None:
    case = inputs.sweep_draws(64, seed=0)[INDEX]
    oracle.set_threads(os.cpu_count() or 1)
    o = oracle.Oracle.from_case(case).init(*case.fields())
    z = {}
    first_bad = None
    for t in range(100, LIMIT + 1, 100):
        o.step(100)
        ob = o.observe()
        if ob["flags"] & 2:
            first_bad = t
            break
        if t % 1000 == 0:
            z[t] = ob["z"]
    out = {"source": "FP64 oracle, tests/golden/make_sweep_instability.py",
           "case": {"sweep_seed": 0, "index": INDEX, "name": case.name, "nx": case.geom.nx, "ny": case.geom.ny,
                    "x0": case.geom.x0, "x1": case.geom.x1, "tau": list(case.params.tau),
                    "gw": list(case.params.gw), "noise_seed": case.seed},
           "sample_every": 100, "first_unstable_t": first_bad, "z_every_1000": {str(k): v for k, v in z.items()}}
    with open(os.path.join(HERE, "sweep_instability_H20_L512_r2.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(first_bad)


if __name__ == "__main__":
    main()
