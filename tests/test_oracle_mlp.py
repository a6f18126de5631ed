"""Pins of the FP64 surrogate reference (oracle/mlp.py).

* gradients against central finite differences (relative error <= 1e-6);
* a one-unit network written out by hand (forward and gradient);
* the first Adam step from zero moments equals lr * g / (|g| + eps) in closed form;
* parameter counts of the 4- and 5-input networks (4 x 256 hidden, 2 outputs);
* the committed trained weights are well formed (shapes, finite values, normalisation).
"""
import math

import numpy as np
import pytest

from oracle import mlp


def test_parameter_counts():
    assert mlp.n_params(4) == 199170
    assert mlp.n_params(5) == 199426


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    d_in, width, depth = 4, 8, 2
    n = mlp.n_params(d_in, width, depth)
    theta = rng.normal(0, 0.5, n)
    X = rng.normal(size=(7, d_in)); T = rng.normal(size=(7, 2)); w = rng.uniform(0.5, 2.0, 7)
    loss, g = mlp.loss_and_grad(theta, X, T, w, d_in, width, depth)
    h = 1e-6
    for j in rng.choice(n, 60, replace=False):
        tp = theta.copy(); tp[j] += h
        tm = theta.copy(); tm[j] -= h
        fd = (mlp.loss_and_grad(tp, X, T, w, d_in, width, depth)[0]
              - mlp.loss_and_grad(tm, X, T, w, d_in, width, depth)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), (j, fd, g[j])


def test_one_unit_network_by_hand():
    # d_in = 1, one hidden unit, one hidden layer: y_o = v_o silu(a x + c) + e_o
    a, c = 0.7, -0.2
    v = np.array([1.5, -0.5]); e = np.array([0.1, 0.3])
    theta = np.array([a, c, v[0], v[1], e[0], e[1]])
    x, t, wt = 0.9, np.array([1.0, 0.0]), 2.0
    z = a * x + c
    s = 1 / (1 + math.exp(-z))
    h = z * s
    y = v * h + e
    Y, _, _ = mlp.forward(theta, np.array([[x]]), 1, width=1, depth=1)
    np.testing.assert_allclose(Y[0], y, rtol=1e-15)
    loss, g = mlp.loss_and_grad(theta, np.array([[x]]), t[None], np.array([wt]), 1, width=1, depth=1)
    r = y - t
    assert abs(loss - 0.5 * wt * (r @ r)) < 1e-15
    dh = wt * (r @ v)
    dz = dh * (s + z * s * (1 - s))
    np.testing.assert_allclose(g, [dz * x, dz, wt * r[0] * h, wt * r[1] * h, wt * r[0], wt * r[1]],
                               rtol=1e-13)


def test_first_adam_step_closed_form():
    g = np.array([0.3, -2.0, 1e-9, 0.0])
    th, m, v = mlp.adam_update(np.zeros(4), g, np.zeros(4), np.zeros(4), step=1, lr=1e-3, eps=1e-8)
    np.testing.assert_allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(m, 0.1 * g); np.testing.assert_allclose(v, 0.001 * g * g)


@pytest.mark.parametrize("d_in", [4, 5])
def test_committed_weights_are_well_formed(d_in):
    """The trained weights shipped with the package: the network of 4 hidden layers of 256 SiLU
    units (199 170 or 199 426 parameters), finite values, a usable input normalisation, a finite
    FP64 forward pass inside the training box, and the training record stored with them."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_0807_0602_amd",
                        f"surrogate_weights_{d_in}in.npz")
    z = np.load(path, allow_pickle=False)
    assert int(z["d_in"]) == d_in and int(z["width"]) == 256 and int(z["depth"]) == 4
    assert z["theta"].shape == (mlp.n_params(d_in),) == ({4: 199170, 5: 199426}[d_in],)
    assert np.isfinite(z["theta"]).all()
    assert (z["std"] > 0).all() and (z["lo"] < z["hi"]).all()
    rng = np.random.default_rng(0)
    X = z["lo"] + (z["hi"] - z["lo"]) * rng.random((64, d_in))
    with np.errstate(over="ignore"):   # exp(-z) of a large negative pre-activation: SiLU(z) = -0
        Y, _, _ = mlp.forward(z["theta"], (X - z["mean"]) / z["std"], d_in)
    assert Y.shape == (64, 2) and np.isfinite(Y).all()
    info = json.loads(str(z["info"]))
    assert info["heldout_channels"] == 200 and 0.0 <= info["heldout_frac_le_1lu"] <= 1.0
