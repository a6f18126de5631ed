"""Macroscopic read-outs of the FP64 model used by the physics pins (test infrastructure only).

  * pressure: Sec. 2 gives p = c0^2 sum_k n_k + (3/2) sum_{k,kbar} g_{k kbar} psi_k psi_kbar
    with c0^2 = 1/3.  With the interaction written as G times the D2Q9 weights, g = G/9 and
    only the two cross terms survive, so p = (n_A + n_B)/3 + (G/3) n_A n_B.
  * mixture velocity (Chapman-Enskog limit, eq. NS): rho u = sum_k rho_k u_k + (1/2) sum_k F_k.
  * dynamic viscosity: mu = sum_k rho_k nu_k with nu_k = (tau_k - 1/2)/3 (Sec. 2).
"""
from __future__ import annotations

import numpy as np


def pressure(nA, nB, G: float = 0.9):
    nA = np.asarray(nA); nB = np.asarray(nB)
    return (nA + nB) / 3.0 + (G / 3.0) * nA * nB


def kinematic_viscosity(tau: float) -> float:
    return (tau - 0.5) / 3.0


def mixture_velocity(macro: dict, mass=(1.0, 1.0)):
    """(ux, uy, rho) of eq. NS from an Oracle.macro() dictionary."""
    n, j, F = macro["n"], macro["j"], macro["F"]
    rho = mass[0] * n[0] + mass[1] * n[1]
    px = mass[0] * j[0, 0] + mass[1] * j[1, 0] + 0.5 * (F[0, 0] + F[1, 0])
    py = mass[0] * j[0, 1] + mass[1] * j[1, 1] + 0.5 * (F[0, 1] + F[1, 1])
    with np.errstate(invalid="ignore", divide="ignore"):
        return px / rho, py / rho, rho


def droplet_radius(nA, level_in: float, level_out: float) -> float:
    """Equivalent radius of a 2-D drop: area = sum of the normalised liquid fraction."""
    frac = (np.asarray(nA) - level_out) / (level_in - level_out)
    return float(np.sqrt(frac.sum() / np.pi))

