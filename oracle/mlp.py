"""FP64 reference of the surrogate network (test infrastructure only).

A multilayer perceptron with `d_in` inputs, `depth` hidden layers of `width` SiLU units and 2
linear outputs, trained on an output-weighted mean squared error with Adam:

    Z_1 = X W_1^T + b_1,  H_l = silu(Z_l),  Z_{l+1} = H_l W_{l+1}^T + b_{l+1},
    Y = H_depth W_out^T + b_out,
    loss = (1 / (2B)) sum_b w_b sum_o (Y_bo - T_bo)^2,          silu(z) = z / (1 + e^{-z}).

The gradients are written out by the chain rule, layer by layer; Adam is the published update
(Kingma and Ba, 2015) with bias correction.  Parameters are a flat float64 vector in the order
W_1, b_1, W_2, b_2, ..., W_out, b_out, each W row-major (out x in) — the same order the HIP
library uses for scf_sur_get_params / scf_sur_set_params.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def layer_shapes(d_in: int, width: int = 256, depth: int = 4, d_out: int = 2) -> List[Tuple[int, int]]:
    dims = [d_in] + [width] * depth + [d_out]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def n_params(d_in: int, width: int = 256, depth: int = 4, d_out: int = 2) -> int:
    return sum(o * i + o for o, i in layer_shapes(d_in, width, depth, d_out))


def unpack(theta: np.ndarray, d_in: int, width: int = 256, depth: int = 4, d_out: int = 2):
    out, p = [], 0
    for o, i in layer_shapes(d_in, width, depth, d_out):
        W = theta[p:p + o * i].reshape(o, i); p += o * i
        b = theta[p:p + o]; p += o
        out.append((W, b))
    assert p == theta.size
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_prime(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X, d_in, width=256, depth=4):
    layers = unpack(np.asarray(theta, np.float64), d_in, width, depth)
    H = np.asarray(X, np.float64)
    Zs, Hs = [], [H]
    for W, b in layers[:-1]:
        Z = H @ W.T + b
        H = silu(Z)
        Zs.append(Z); Hs.append(H)
    W, b = layers[-1]
    return H @ W.T + b, Zs, Hs


def loss_and_grad(theta, X, T, w, d_in, width=256, depth=4):
    """Loss and its gradient with respect to the flat parameter vector."""
    layers = unpack(np.asarray(theta, np.float64), d_in, width, depth)
    Y, Zs, Hs = forward(theta, X, d_in, width, depth)
    B = X.shape[0]
    w = np.asarray(w, np.float64).reshape(B, 1)
    R = Y - T
    loss = 0.5 * float((w * R * R).sum()) / B
    dY = w * R / B
    grads = [None] * len(layers)
    W, _ = layers[-1]
    grads[-1] = (dY.T @ Hs[-1], dY.sum(axis=0))
    dH = dY @ W
    for l in range(len(layers) - 2, -1, -1):
        dZ = dH * silu_prime(Zs[l])
        grads[l] = (dZ.T @ Hs[l], dZ.sum(axis=0))
        if l > 0:
            dH = dZ @ layers[l][0]
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_update(theta, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
