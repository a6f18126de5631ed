"""Front dynamics of the capillary-filling experiment (test infrastructure only).

Sec. 2.1 of the paper balances the momentum of liquid plus gas inside a capillary of length
L and height H (eq. momentum) with a Poiseuille profile, giving the front equation (eq. GWE):

    (rho_g (L - z) + rho_l z) z'' + (rho_l - rho_g) z'^2
        = 2 gamma cos(theta) / H - (12 z' / H^2) (mu_g (L - z) + mu_l z)

This module integrates it with the classical fourth-order Runge-Kutta method (the paper used
Mathematica), and states its closed-form limits:
  * eq. analy:   rho_l = rho_g, mu_l = mu_g  ->  z(t) = (gamma H cos / (6 mu L)) t_d
                 (exp(-t/t_d) + t/t_d - 1) + z0,  t_d = rho H^2 / (12 mu)
  * eq. wash:    no inertia, mu_g -> 0        ->  z^2 - z0^2 = gamma H cos t / (3 mu)
  * no inertia, mu_g > 0 (the viscosity-ratio correction of Sec. 2.1):
                 (mu_l - mu_g)(z^2 - z0^2)/2 + mu_g L (z - z0) = gamma H cos (t - t0) / 6
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class FrontParams:
    gamma: float      # liquid-gas surface tension
    cos_theta: float  # static contact angle
    H: float          # channel height
    L: float          # capillary length
    rho_l: float
    rho_g: float
    mu_l: float
    mu_g: float


def gwe_accel(z: float, v: float, p: FrontParams) -> float:
    """z'' from eq. GWE."""
    mass = p.rho_g * (p.L - z) + p.rho_l * z
    force = 2.0 * p.gamma * p.cos_theta / p.H - (12.0 * v / p.H ** 2) * (p.mu_g * (p.L - z) + p.mu_l * z)
    return (force - (p.rho_l - p.rho_g) * v * v) / mass


def integrate_gwe(p: FrontParams, z0: float, v0: float, t: np.ndarray, dt: float = 0.5) -> np.ndarray:
    """RK4 solution z(t) of eq. GWE sampled at the (increasing, >= 0) times t."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    z, v, tc = float(z0), float(v0), 0.0
    for m, target in enumerate(t):
        while tc < target - 1e-12:
            h = min(dt, target - tc)
            k1z, k1v = v, gwe_accel(z, v, p)
            k2z, k2v = v + 0.5 * h * k1v, gwe_accel(z + 0.5 * h * k1z, v + 0.5 * h * k1v, p)
            k3z, k3v = v + 0.5 * h * k2v, gwe_accel(z + 0.5 * h * k2z, v + 0.5 * h * k2v, p)
            k4z, k4v = v + h * k3v, gwe_accel(z + h * k3z, v + h * k3v, p)
            z += h / 6.0 * (k1z + 2 * k2z + 2 * k3z + k4z)
            v += h / 6.0 * (k1v + 2 * k2v + 2 * k3v + k4v)
            tc += h
        out[m] = z
    return out


def analytic_equal(t, gamma, H, cos_theta, mu, L, rho, z0=0.0):
    """eq. analy: equal densities and viscosities, starting at rest."""
    t = np.asarray(t, dtype=np.float64)
    td = rho * H * H / (12.0 * mu)
    return gamma * H * cos_theta / (6.0 * mu * L) * td * (np.exp(-t / td) + t / td - 1.0) + z0


def washburn_z2(t, gamma, H, cos_theta, mu, z0=0.0):
    """eq. wash: z^2(t) = z0^2 + gamma H cos t / (3 mu)."""
    return z0 * z0 + gamma * H * cos_theta * np.asarray(t, dtype=np.float64) / (3.0 * mu)


def drag_corrected_lhs(z, z0, mu_l, mu_g, L):
    """Left side of the inertia-free front law with gas drag; equals gamma H cos (t - t0) / 6."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (mu_l - mu_g) * (z * z - z0 * z0) + mu_g * L * (z - z0)
