"""Writes density_ratio_droplets.json with the FP64 oracle (run from the repository root:
python tests/golden/make_density_ratio_droplets.py).

Four static drops of A (radius 10, 14, 18, 22) in periodic 96 x 96 boxes with unequal sound
speeds (rest fractions alpha = (0.8, 4/9), eqs. feq1-feq3), the paper's relaxation times for its
water-in-air runs (tau = 2.5 and 0.626) and G = 1.5, started from n = (1.25, 0.005) inside and
(0.17, 0.31) outside, 20 000 steps.  Recorded per drop: the smallest density of either component
anywhere in the box (the minority component dips slightly below zero in this model, so the GPU
health bound for these drops is the oracle's own minimum), the drop radius from its area
(nodes with n_A > n_B) and the pressure jump p_in - p_out with p = sum_k n_k 3 (1 - alpha_k)/5 +
(G/3) n_A n_B (unit masses), read inside half the radius and outside R + 0.35 (48 - R).
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_0807_0602_amd import inputs  # noqa: E402

N, STEPS, G = 96, 20_000, 1.5
ALPHA, TAU = (0.8, 4.0 / 9.0), (2.5, 0.626)
RADII = (10, 14, 18, 22)


def pressure(nA, nB):
    return nA * 3.0 * (1.0 - ALPHA[0]) / 5.0 + nB * 3.0 * (1.0 - ALPHA[1]) / 5.0 + (G / 3.0) * nA * nB


def main() -> None:
    oracle.set_threads(os.cpu_count() or 1)
    c = (N - 1) / 2.0
    Y, X = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    r = np.hypot(X - c, Y - c)
    drops = []
    for R0 in RADII:
        a, b = inputs.droplet_fields(N, R0, rho_liq=1.25, rho_min=0.005, gas=(0.17, 0.31))
        o = oracle.Oracle(N, N, 0, 0, G, (0.0, 0.0), TAU, alpha=ALPHA, mass=(1.0, 1.0)).init(a, b).step(STEPS)
        nA, nB = o.density()
        R = float(np.sqrt(np.count_nonzero(nA > nB) / np.pi))
        p = pressure(nA, nB)
        dp = float(p[r < 0.5 * R].mean() - p[r > R + 0.35 * (N / 2 - R)].mean())
        drops.append({"R0": R0, "min_density": float(min(nA.min(), nB.min())), "R": R, "dp": dp,
                      "nA_centre": float(nA[N // 2, N // 2]), "nB_far": float(nB[0, 0])})
        print(drops[-1], flush=True)
    out = {"source": "FP64 oracle, tests/golden/make_density_ratio_droplets.py", "n": N, "steps": STEPS,
           "G": G, "alpha": list(ALPHA), "tau": list(TAU), "init_inside": [1.25, 0.005],
           "init_outside": [0.17, 0.31], "drops": drops}
    with open(os.path.join(HERE, "density_ratio_droplets.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
