"""GPU surrogate network (scf_sur_*) against the FP64 reference in oracle/mlp.py.

The hidden layers run in BF16 on MFMA with FP32 accumulation, so results match the FP64
reference to BF16 accuracy: outputs to a few 1e-2 relative, gradients with cosine similarity
> 0.999 and relative L2 error < 2e-2 per parameter block.  Adam's first step from zero moments is
-lr * g / (|g| + eps), so its sign and size are checked against the reference gradient.
"""
import sys

import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu

D_IN, WIDTH, DEPTH = 4, 256, 4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sur():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0807_0602_amd import surrogate
    return surrogate


def _random_theta(seed, d_in=D_IN, width=WIDTH, depth=DEPTH):
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in mlp.layer_shapes(d_in, width, depth):
        parts.append(rng.normal(0, 1.0 / np.sqrt(i), o * i))
        parts.append(rng.normal(0, 0.3, o))
    return np.concatenate(parts)


def _problem(seed, n, d_in=D_IN):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d_in))
    T = rng.normal(0, 0.5, size=(n, 2))
    w = rng.uniform(0.5, 2.0, n)
    return X, T, w


def _blocks(d_in=D_IN, width=WIDTH, depth=DEPTH):
    out, p = [], 0
    for l, (o, i) in enumerate(mlp.layer_shapes(d_in, width, depth)):
        out.append((f"W{l}", slice(p, p + o * i))); p += o * i
        out.append((f"b{l}", slice(p, p + o))); p += o
    return out


def test_parameter_count_and_init(sur):
    net = sur.Network(D_IN, WIDTH, DEPTH, max_batch=256, max_data=1024, seed=1)
    assert net.n_params == mlp.n_params(D_IN, WIDTH, DEPTH) == 199170
    th = net.params()
    for name, sl in _blocks():
        v = th[sl]
        if name.startswith("b"):
            assert np.all(v == 0)
        else:
            fan_in = D_IN if name == "W0" else WIDTH
            assert np.abs(v).max() <= 1.0 / np.sqrt(fan_in) + 1e-7 and v.std() > 0.4 / np.sqrt(fan_in)
    net2 = sur.Network(D_IN, WIDTH, DEPTH, max_batch=256, max_data=1024, seed=1)
    assert np.array_equal(th, net2.params())


def test_forward_matches_oracle(sur):
    _say("case: surrogate forward vs FP64, 200 rows")
    net = sur.Network(D_IN, WIDTH, DEPTH, max_batch=512, max_data=1024, seed=2)
    theta = _random_theta(7)
    net.set_params(theta.astype(np.float32))
    X, _, _ = _problem(3, 200)
    Y, _ = net.predict(X)
    Yo, _, _ = mlp.forward(theta.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64), D_IN)
    rel = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    _say(f"  rel L2 = {rel:.3e}")
    assert rel < 3e-2
    assert np.corrcoef(Y.ravel(), Yo.ravel())[0, 1] > 0.999


@pytest.mark.parametrize("n", [64, 200, 1000])
def test_gradients_match_oracle(sur, n):
    _say(f"case: surrogate gradients vs FP64, {n} rows")
    net = sur.Network(D_IN, WIDTH, DEPTH, max_batch=1024, max_data=1024, seed=2)
    theta = _random_theta(11).astype(np.float32)
    net.set_params(theta)
    X, T, w = _problem(5 + n, n)
    loss, g = net.grad(X, T, w)
    lo, go = mlp.loss_and_grad(theta.astype(np.float64), X.astype(np.float32).astype(np.float64),
                               T.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64), D_IN)
    assert abs(loss - lo) / lo < 2e-2
    for name, sl in _blocks():
        a, b = g[sl].astype(np.float64), go[sl]
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        _say(f"  {name}: cos = {cos:.6f} rel = {rel:.2e}")
        assert cos > 0.999 and rel < 2e-2, name


def test_first_adam_step(sur):
    _say("case: first Adam step")
    lr = 1e-3
    net = sur.Network(D_IN, WIDTH, DEPTH, max_batch=512, max_data=1024, lr=lr, seed=2)
    theta = _random_theta(13).astype(np.float32)
    net.set_params(theta)
    net.reset_optimizer()
    X, T, w = _problem(17, 300)
    net.step(X, T, w)
    delta = net.params().astype(np.float64) - theta.astype(np.float64)
    _, go = mlp.loss_and_grad(theta.astype(np.float64), X.astype(np.float32).astype(np.float64),
                              T.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64), D_IN)
    big = np.abs(go) > 1e-3 * np.abs(go).max()
    expect = -lr * go / (np.abs(go) + 1e-8)
    agree = np.mean(np.sign(delta[big]) == np.sign(expect[big]))
    _say(f"  sign agreement {agree:.5f} on {big.sum()} parameters")
    assert agree > 0.99
    # |delta| = lr up to the FP32 rounding of theta +- lr
    np.testing.assert_allclose(np.abs(delta[big]), lr, rtol=0, atol=lr * 2e-3 + 1e-6)


def test_training_reduces_loss_and_is_deterministic(sur):
    _say("case: training on a smooth synthetic map")
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, size=(8192, D_IN)).astype(np.float32)
    T = np.stack([np.sin(2 * X[:, 0] + X[:, 1]), X[:, 2] * X[:, 3]], axis=1).astype(np.float32)
    nets = []
    for _ in range(2):
        net = sur.Network(D_IN, WIDTH, DEPTH, max_batch=1024, max_data=8192, lr=1e-3, seed=5)
        net.set_data(X, T)
        first = net.train(1, 1024)
        last = net.train(400, 1024)
        nets.append((net, first, last))
    (a, first, last), (b, _, last_b) = nets
    _say(f"  loss {first:.4f} -> {last:.5f}")
    assert last < 0.1 * first
    assert last == last_b and np.array_equal(a.params(), b.params())
    # the trained map generalises to fresh points
    Xt = rng.uniform(-1, 1, size=(512, D_IN)).astype(np.float32)
    Tt = np.stack([np.sin(2 * Xt[:, 0] + Xt[:, 1]), Xt[:, 2] * Xt[:, 3]], axis=1)
    Y, inside = a.predict(Xt)
    assert inside.mean() > 0.95
    assert np.sqrt(np.mean((Y - Tt) ** 2)) < 0.1


def test_normalisation_and_hull(sur):
    net = sur.Network(D_IN, WIDTH, DEPTH, max_batch=256, max_data=4096, seed=1)
    rng = np.random.default_rng(1)
    X = np.stack([rng.uniform(-0.3, 0.3, 4000), rng.choice([0.0, -0.4, -0.9], 4000),
                  rng.uniform(20, 160, 4000), rng.uniform(np.log(100), np.log(5e4), 4000)], axis=1).astype(np.float32)
    T = np.zeros((4000, 2), np.float32)
    net.set_data(X, T)
    st = net.norm()
    np.testing.assert_allclose(st["mean"], X.astype(np.float64).mean(axis=0), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(st["std"], X.astype(np.float64).std(axis=0), rtol=1e-4)
    np.testing.assert_array_equal(st["lo"], X.min(axis=0))
    np.testing.assert_array_equal(st["hi"], X.max(axis=0))
    Q = np.array([X[0], X[1] * [1, 1, 1, 1], [0.5, 0.0, 50, 8.0], [0.0, 0.0, 10.0, 8.0], [0.0, -0.4, 100, 20.0]],
                 np.float32)
    _, inside = net.predict(Q)
    assert list(inside) == [True, True, False, False, False]
