"""Surrogate of the batched LBM: a network from sweep parameters and time to the front and
precursor positions, trained on the GPU by the library's own MFMA kernels (scf_sur_* in
include/scf.h), with the LBM as fallback outside the training range and as judge of its error.

Features of one sample (A-S1 of the design notes: the 4-input set, optionally the channel
length): (G_wA, log(tau_B / tau_A), H, log t[, log L]).  Targets: (z / H, p / H).  Sample
weight H^2, so the loss is the squared error in lattice units.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L
from .inputs import Case


def _fp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def features(case: Case, t, with_length: bool = False) -> np.ndarray:
    """Input rows for one channel at times t (array)."""
    t = np.asarray(t, dtype=np.float64)
    p, g = case.params, case.geom
    cols = [np.full_like(t, p.gw[0]), np.full_like(t, math.log(p.tau[1] / p.tau[0])),
            np.full_like(t, float(g.ny - 2)), np.log(t)]
    if with_length:
        cols.append(np.full_like(t, math.log(float(g.x1 - g.x0))))
    return np.stack(cols, axis=1).astype(np.float32)


class Network:
    """One surrogate network in a device workspace (scf_sur_create ... scf_sur_destroy)."""

    def __init__(self, d_in: int = 4, width: int = 256, depth: int = 4, max_batch: int = 4096,
                 max_data: int = 1 << 20, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, seed: int = 0, device="cuda:0",
                 stream: Optional[torch.cuda.Stream] = None):
        self.cfg = L.scf_sur_cfg(d_in, width, depth, max_batch, max_data, lr, beta1, beta2, eps, seed)
        nbytes = L.scf_sur_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise L.ScfError(L.SCF_EINVAL, "invalid surrogate configuration")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        s = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        L.check(L.scf_sur_create(C.byref(h), C.byref(self.cfg), C.c_void_p(self.ws.data_ptr()), nbytes,
                                 C.c_void_p(s.cuda_stream)))
        self._h = h
        self.n_params = int(L.scf_sur_param_count(h))

    def close(self):
        if getattr(self, "_h", None) and getattr(L, "scf_sur_destroy", None) is not None:
            L.scf_sur_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        L.check(L.scf_sur_get_params(self._h, _fp(out)))
        return out

    def set_params(self, theta: np.ndarray) -> None:
        a = np.ascontiguousarray(theta, np.float32)
        assert a.size == self.n_params
        L.check(L.scf_sur_set_params(self._h, _fp(a)))

    def reset_optimizer(self) -> None:
        L.check(L.scf_sur_reset_optimizer(self._h))

    def set_data(self, X: np.ndarray, T: np.ndarray, w: Optional[np.ndarray] = None) -> None:
        X = np.ascontiguousarray(X, np.float32); T = np.ascontiguousarray(T, np.float32)
        wp = None
        if w is not None:
            w = np.ascontiguousarray(w, np.float32); wp = _fp(w)
        L.check(L.scf_sur_set_data(self._h, _fp(X), _fp(T), wp, X.shape[0]))

    def norm(self) -> dict:
        d = self.cfg.d_in
        out = {k: np.empty(d, np.float32) for k in ("mean", "std", "lo", "hi")}
        L.check(L.scf_sur_get_norm(self._h, _fp(out["mean"]), _fp(out["std"]), _fp(out["lo"]), _fp(out["hi"])))
        return out

    def grad(self, X, T, w=None) -> Tuple[float, np.ndarray]:
        X = np.ascontiguousarray(X, np.float32); T = np.ascontiguousarray(T, np.float32)
        wp = None
        if w is not None:
            w = np.ascontiguousarray(w, np.float32); wp = _fp(w)
        loss = np.zeros(1, np.float32); g = np.empty(self.n_params, np.float32)
        L.check(L.scf_sur_grad(self._h, _fp(X), _fp(T), wp, X.shape[0], _fp(loss), _fp(g)))
        return float(loss[0]), g

    def step(self, X, T, w=None) -> float:
        X = np.ascontiguousarray(X, np.float32); T = np.ascontiguousarray(T, np.float32)
        wp = None
        if w is not None:
            w = np.ascontiguousarray(w, np.float32); wp = _fp(w)
        loss = np.zeros(1, np.float32)
        L.check(L.scf_sur_step(self._h, _fp(X), _fp(T), wp, X.shape[0], _fp(loss)))
        return float(loss[0])

    def train(self, steps: int, batch: int = 4096) -> float:
        loss = np.zeros(1, np.float32)
        L.check(L.scf_sur_train(self._h, int(steps), int(batch), _fp(loss)))
        return float(loss[0])

    def predict(self, X) -> Tuple[np.ndarray, np.ndarray]:
        X = np.ascontiguousarray(X, np.float32)
        n = X.shape[0]
        Y = np.empty((n, 2), np.float32); inside = np.empty(n, np.uint8)
        L.check(L.scf_sur_predict(self._h, _fp(X), n, _fp(Y), inside.ctypes.data_as(C.POINTER(C.c_uint8))))
        return Y, inside.astype(bool)
