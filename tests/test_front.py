"""The front equation (eq. GWE) integrator against the paper's closed forms.

  * equal densities and viscosities: eq. analy, exactly;
  * no gas (rho_g = mu_g = 0), start at rest: z^2 - z0^2 = (gamma H cos / 3 mu)
    (t - t_d (1 - exp(-t/t_d))) with t_d = rho H^2 / (12 mu), which tends to eq. wash;
  * inertia-free limit with gas drag: (mu_l - mu_g)(z^2 - z0^2)/2 + mu_g L (z - z0) grows at
    gamma H cos / 6 at late times.
"""
import numpy as np

from oracle import front


def test_rk4_matches_eq_analy():
    p = front.FrontParams(gamma=0.18, cos_theta=0.4, H=22, L=100, rho_l=2.0, rho_g=2.0,
                          mu_l=2.0 / 6, mu_g=2.0 / 6)
    t = np.linspace(0, 3000, 31)
    z = front.integrate_gwe(p, z0=-0.5, v0=0.0, t=t, dt=0.5)
    ref = front.analytic_equal(t, 0.18, 22, 0.4, 2.0 / 6, 100, 2.0, z0=-0.5)
    np.testing.assert_allclose(z, ref, rtol=0, atol=1e-9)


def test_rk4_no_gas_closed_form_and_washburn_limit():
    g, c, H, mu, rho = 0.18, 0.7, 40.0, 0.5, 2.0
    p = front.FrontParams(gamma=g, cos_theta=c, H=H, L=1000, rho_l=rho, rho_g=0.0, mu_l=mu, mu_g=0.0)
    z0 = 5.0
    t = np.array([0.0, 100, 500, 2000, 20000, 200000])
    z = front.integrate_gwe(p, z0=z0, v0=0.0, t=t, dt=0.25)
    td = rho * H * H / (12 * mu)
    ref = z0 ** 2 + g * H * c / (3 * mu) * (t - td * (1 - np.exp(-t / td)))
    np.testing.assert_allclose(z ** 2, ref, rtol=1e-8, atol=1e-8)
    # late times: eq. wash up to the constant inertial lag t_d
    w = front.washburn_z2(t[-1] - td, g, H, c, mu, z0)
    assert abs(z[-1] ** 2 - w) / w < 1e-9


def test_drag_corrected_law_late_slope():
    g, c, H, L = 0.18, 0.5, 40.0, 600.0
    mu_l, mu_g = 0.8, 0.08
    p = front.FrontParams(gamma=g, cos_theta=c, H=H, L=L, rho_l=2.0, rho_g=0.06, mu_l=mu_l, mu_g=mu_g)
    t = np.linspace(20000, 60000, 9)
    z = front.integrate_gwe(p, z0=0.0, v0=0.0, t=t, dt=1.0)
    lhs = front.drag_corrected_lhs(z, 0.0, mu_l, mu_g, L)
    slope = np.polyfit(t, lhs, 1)[0]
    assert abs(slope / (g * H * c / 6.0) - 1.0) < 1e-3
