"""Surrogate of the batched LBM: a network from sweep parameters and time to the front and
precursor positions, trained on the GPU by the library's own MFMA kernels (scf_sur_* in
include/scf.h), with the LBM as fallback outside the training range and as the reference for its error.

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

    def set_lr(self, lr: float) -> None:
        L.check(L.scf_sur_set_lr(self._h, float(lr)))

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

    def set_norm(self, mean, std, lo, hi) -> None:
        a = [np.ascontiguousarray(v, np.float32) for v in (mean, std, lo, hi)]
        L.check(L.scf_sur_set_norm(self._h, *[_fp(v) for v in a]))

    def save(self, path: str, **extra) -> None:
        n = self.norm()
        c = self.cfg
        np.savez(path, theta=self.params(), mean=n["mean"], std=n["std"], lo=n["lo"], hi=n["hi"],
                 d_in=c.d_in, width=c.width, depth=c.depth, **extra)

    @classmethod
    def load(cls, path: str, max_batch: int = 4096, **kw) -> "Network":
        z = np.load(path)
        net = cls(int(z["d_in"]), int(z["width"]), int(z["depth"]), max_batch=max_batch, max_data=64, **kw)
        net.set_params(z["theta"])
        net.set_norm(z["mean"], z["std"], z["lo"], z["hi"])
        return net

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


# ---------------------------------------------------------------------------------------------
# Data from the batched LBM, training, evaluation and the LBM fallback.
# ---------------------------------------------------------------------------------------------

RATIOS = (1, 2, 5, 10)


def draw_cases(n: int, seed: int, steps: int = 50_000, every: int = 100, grid: bool = False) -> List[Case]:
    """n channels with G_wA ~ U[-0.3, 0.3], H ~ U{20..160}, L ~ U{512..4096} in multiples of 4
    and r uniform over {1, 2, 5, 10} (tau pair per the working map of inputs.TAU_FOR_RATIO).
    grid: H and L uniform over the calibration sweep's own sets instead, {20, 40, 80, 160} and
    {512, 1024, 2048, 4096} (the sweep recipe inputs.sweep_draws with this seed)."""
    from .inputs import sweep_channel, sweep_draws
    if grid:
        return sweep_draws(n, seed=seed, steps=steps, sample_every=every)
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n):
        H = int(rng.integers(20, 161))
        L_ = 4 * int(rng.integers(128, 1025))
        r = int(rng.choice(RATIOS))
        g = float(rng.uniform(-0.3, 0.3))
        out.append(sweep_channel(H, L_, g, r, seed=100_000 * (seed + 1) + c, steps=steps, sample_every=every))
    return out


def simulate(cases: Sequence[Case], steps: int, every: int, group: int = 64, log=None) -> np.ndarray:
    """Trajectories of every channel from the batched LBM, `group` channels per batch.
    Returns float64 [n, steps/every + 1, 5]: t, z, precursor, flags, unstable-so-far."""
    from .scf import Batch
    ns = steps // every + 1
    out = np.full((len(cases), ns, 5), np.nan)
    for g0 in range(0, len(cases), group):
        part = list(cases[g0:g0 + group])
        b = Batch(part, sample_every=every, max_samples=ns)
        b.set_tile(256, 16, every, 6, 2)   # persistent, two steps per launch (the sweep's autotuned schedule)
        b.step(steps)
        recs, k = b.observe(allow_unstable=True)
        for c, r in enumerate(recs):
            bad = False
            for s, x in enumerate(r):
                bad = bad or bool(x["flags"] & 2)
                out[g0 + c, s] = (x["t"], x["z"], x["precursor"], x["flags"], float(bad))
        b.close()
        if log:
            log(f"simulated channels {g0}..{g0 + len(part) - 1}")
    return out


def precursor_jumped(t: np.ndarray, p: np.ndarray) -> np.ndarray:
    """True from the first sample at which the precursor moved farther than one node per step
    since the previous sample where it was found (missing samples are skipped).  No front moves
    faster than the lattice speed; such a jump is the precursor level (a third of the liquid
    reservoir's density at its centre) dropping as the reservoir drains, one sample before the
    drain flag, when the crossing search leaps to the far end of the channel."""
    t = np.asarray(t, np.float64)
    p = np.asarray(p, np.float64)
    i = np.nonzero(np.isfinite(p))[0]
    jump = np.zeros(p.shape, bool)
    if i.size > 1:
        jump[i[1:]] = np.abs(np.diff(p[i])) > np.diff(t[i])
    return np.cumsum(jump) > 0


def dataset(cases: Sequence[Case], traj: np.ndarray, with_length: bool = False, t_min: float = 100.0):
    """(X, T, w, keep): features, targets (z/H, p/H), weights H^2, and the mask of kept samples
    (t >= t_min, finite z and p, no instability so far, and the liquid reservoir not yet drained:
    from the drain flag on (the reservoir drained to its centre) the film level is read in gas and
    the front is no longer fed by a reservoir, so the samples no longer describe capillary
    filling; the drain shows one sample earlier as a precursor jump faster than the lattice
    speed, see precursor_jumped)."""
    Xs, Ts, ws, keep = [], [], [], []
    for case, tr in zip(cases, traj):
        H = float(case.geom.ny - 2)
        t, z, p, flags, unst = tr[:, 0], tr[:, 1], tr[:, 2], tr[:, 3], tr[:, 4]
        drained = (np.cumsum((np.nan_to_num(flags).astype(np.int64) & 1) > 0) > 0) | precursor_jumped(t, p)
        ok = (t >= t_min) & np.isfinite(z) & np.isfinite(p) & (unst == 0) & ~drained
        Xs.append(features(case, np.maximum(t, 1.0), with_length))
        Ts.append(np.stack([z / H, p / H], axis=1))
        ws.append(np.full(t.shape, H * H))
        keep.append(ok)
    X = np.concatenate(Xs).astype(np.float32)
    T = np.concatenate(Ts).astype(np.float32)
    w = np.concatenate(ws).astype(np.float32)
    k = np.concatenate(keep)
    return X, T, w, k


def curve_errors(net: Network, cases: Sequence[Case], traj: np.ndarray, with_length: bool = False):
    """Per-channel max |z_surrogate - z_LBM| and max |p_surrogate - p_LBM| in lattice units over the
    kept samples, and the fraction of samples inside the training hull."""
    X, T, w, k = dataset(cases, traj, with_length)
    Y, inside = net.predict(X)
    ns = traj.shape[1]
    errs = []
    for c, case in enumerate(cases):
        H = float(case.geom.ny - 2)
        sl = slice(c * ns, (c + 1) * ns)
        m = k[sl]
        if not m.any():
            errs.append((np.nan, np.nan))
            continue
        dz = np.abs(Y[sl][m, 0] - T[sl][m, 0]) * H
        dp = np.abs(Y[sl][m, 1] - T[sl][m, 1]) * H
        errs.append((float(dz.max()), float(dp.max())))
    return np.array(errs), float(inside[k].mean()) if k.any() else 0.0


def predict_curves(net: Network, cases: Sequence[Case], t: np.ndarray, with_length: bool = False,
                   every: int = 100):
    """z(t), p(t) for each channel at times t: the network inside the training hull, the batched
    LBM for channels with any query outside it (the fallback).  Returns (Z, P, used_lbm)."""
    t = np.asarray(t, dtype=np.float64)
    Z = np.empty((len(cases), t.size)); P = np.empty_like(Z)
    outside = []
    for c, case in enumerate(cases):
        Y, inside = net.predict(features(case, t, with_length))
        H = float(case.geom.ny - 2)
        Z[c], P[c] = Y[:, 0] * H, Y[:, 1] * H
        if not inside.all():
            outside.append(c)
    if outside:
        steps = int(math.ceil(t.max() / every) * every)
        traj = simulate([cases[c] for c in outside], steps, every)
        for j, c in enumerate(outside):
            idx = np.clip(np.rint(t / every).astype(int), 0, traj.shape[1] - 1)
            Z[c], P[c] = traj[j, idx, 1], traj[j, idx, 2]
    used = np.zeros(len(cases), bool); used[outside] = True
    return Z, P, used


# ---------------------------------------------------------------------------------------------
# Command line: generate trajectories, train, evaluate.
#   python -m paper_0807_0602_amd.surrogate generate --n 1000 --seed 1 --out train1.npz
#   python -m paper_0807_0602_amd.surrogate train --data train1.npz train2.npz --inputs 5 --out w.npz
#   python -m paper_0807_0602_amd.surrogate evaluate --weights w.npz --data heldout.npz
# ---------------------------------------------------------------------------------------------

def save_trajectories(path: str, cases: Sequence[Case], traj: np.ndarray, steps: int, every: int,
                      seconds: float = float("nan")) -> None:
    """Trajectories with their channel parameters and the GPU seconds the LBM took for them."""
    from .inputs import TAU_FOR_RATIO
    ratio_of = {tau: r for r, tau in TAU_FOR_RATIO.items()}
    meta = np.array([(c.geom.ny - 2, c.geom.x1 - c.geom.x0, c.params.gw[0], ratio_of[tuple(c.params.tau)], c.seed)
                     for c in cases], dtype=np.float64)
    np.savez_compressed(path, meta=meta, traj=traj.astype(np.float32), steps=steps, every=every,
                        seconds=float(seconds))


def trajectory_seconds(path: str) -> float:
    """The LBM seconds stored with a trajectory file (NaN if it has none)."""
    z = np.load(path)
    return float(z["seconds"]) if "seconds" in z.files else float("nan")


def load_trajectories(path: str):
    from .inputs import sweep_channel
    z = np.load(path)
    steps, every = int(z["steps"]), int(z["every"])
    cases = [sweep_channel(int(H), int(L_), float(g), int(r), seed=int(sd), steps=steps, sample_every=every)
             for H, L_, g, r, sd in z["meta"]]
    return cases, z["traj"].astype(np.float64)


def _main(argv=None) -> int:
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser(prog="python -m paper_0807_0602_amd.surrogate")
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--n", type=int, required=True); g.add_argument("--seed", type=int, required=True)
    g.add_argument("--steps", type=int, default=50_000); g.add_argument("--every", type=int, default=100)
    g.add_argument("--group", type=int, default=64); g.add_argument("--out", required=True)
    g.add_argument("--grid", action="store_true", help="H and L from the sweep's sets")
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True); t.add_argument("--inputs", type=int, choices=[4, 5], default=5)
    t.add_argument("--steps", type=int, default=20_000); t.add_argument("--batch", type=int, default=4096)
    t.add_argument("--lr", type=float, default=1e-3); t.add_argument("--seed", type=int, default=0)
    t.add_argument("--heldout", default=None); t.add_argument("--out", required=True)
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", required=True); e.add_argument("--data", required=True)
    a = ap.parse_args(argv)
    say = lambda m: print(m, flush=True)
    if a.cmd == "generate":
        cases = draw_cases(a.n, a.seed, a.steps, a.every, grid=a.grid)
        t0 = time.perf_counter()
        traj = simulate(cases, a.steps, a.every, a.group, log=say)
        dt = time.perf_counter() - t0
        save_trajectories(a.out, cases, traj, a.steps, a.every, seconds=dt)
        unstable = int((traj[:, -1, 4] > 0).sum())
        say(json.dumps({"generated": a.n, "seconds": round(dt, 1), "unstable": unstable, "out": a.out}))
        return 0
    if a.cmd == "train":
        cases, trajs = [], []
        for p in a.data:
            c, tr = load_trajectories(p); cases += c; trajs.append(tr)
        traj = np.concatenate(trajs)
        wl = a.inputs == 5
        X, T, w, k = dataset(cases, traj, wl)
        X, T, w = X[k], T[k], w[k]
        net = Network(a.inputs, 256, 4, max_batch=a.batch, max_data=X.shape[0], lr=a.lr, seed=a.seed)
        net.set_data(X, T, w)
        t0 = time.perf_counter()
        losses = []
        chunk = 1000
        for s0 in range(0, a.steps, chunk):
            # cosine decay of the step size down to 1 % over the run
            frac = s0 / max(1, a.steps)
            net.set_lr(a.lr * (0.01 + 0.99 * 0.5 * (1.0 + math.cos(math.pi * frac))))
            losses.append(net.train(min(chunk, a.steps - s0), a.batch))
            say(f"step {s0 + chunk}: minibatch loss {losses[-1]:.4f} (lattice units^2)")
        dt = time.perf_counter() - t0
        data_s = sum(trajectory_seconds(p) for p in a.data)
        info = {"train_rows": int(X.shape[0]), "train_channels": len(cases), "steps": a.steps, "batch": a.batch,
                "seconds": round(dt, 1), "final_loss": losses[-1],
                "data_seconds": round(data_s, 1) if math.isfinite(data_s) else None}
        if a.heldout:
            hc, ht = load_trajectories(a.heldout)
            errs, inside = curve_errors(net, hc, ht, wl)
            ok = np.isfinite(errs[:, 0])
            info.update({"heldout_channels": int(ok.sum()), "heldout_max_dz": float(np.nanmax(errs[:, 0])),
                         "heldout_median_max_dz": float(np.nanmedian(errs[:, 0])),
                         "heldout_frac_le_1lu": float(np.mean(errs[ok, 0] <= 1.0)), "inside_hull": inside})
        net.save(a.out, info=json.dumps(info))
        say(json.dumps(info))
        return 0
    if a.cmd == "evaluate":
        z = np.load(a.weights)
        net = Network.load(a.weights)
        hc, ht = load_trajectories(a.data)
        errs, inside = curve_errors(net, hc, ht, int(z["d_in"]) == 5)
        ok = np.isfinite(errs[:, 0])
        say(json.dumps({"channels": int(ok.sum()), "max_dz": float(np.nanmax(errs[:, 0])),
                        "median_max_dz": float(np.nanmedian(errs[:, 0])),
                        "frac_le_1lu": float(np.mean(errs[ok, 0] <= 1.0)), "inside_hull": inside}))
        return 0
    return 2


if __name__ == "__main__":
    raise SystemExit(_main())
