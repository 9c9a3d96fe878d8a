"""Pins of the oracle's van der Waals closed forms (oracle/thermo.py) against
values the paper prints and against mathematical identities."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import thermo

with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as fh:
    PAPER = json.load(fh)


def test_maxwell_matches_printed_coexistence_at_T08():
    """Sec. III A/C print rho_V = 0.23967 and rho_L = 1.9327 at T = 0.8."""
    g = PAPER["coexistence_T0.8"]
    rv, rl = thermo.maxwell(0.8)
    assert rv == pytest.approx(g["rho_V_more_digits"], abs=6e-6)
    assert rl == pytest.approx(g["rho_L"], abs=6e-5)


@pytest.mark.parametrize("T", [0.6, 0.8, 0.95, 0.99])
def test_maxwell_equal_area(T):
    """Coexistence by equal pressure and chemical potential equals the
    equal-area rule int_{v_L}^{v_V} (p - p_coex) dv = 0 in the specific volume."""
    rv, rl = thermo.maxwell(T)
    P = thermo.pressure(rv, T)
    assert thermo.pressure(rl, T) == pytest.approx(P, rel=1e-12)
    area, _ = integrate.quad(lambda v: thermo.pressure(1.0 / v, T) - P, 1.0 / rl, 1.0 / rv, limit=400,
                             epsabs=1e-13, epsrel=1e-12)
    assert abs(area) < 1e-9 * P * (1.0 / rv - 1.0 / rl)
    assert rv < 1.0 < rl  # rho_c = 1 in the paper's units


def test_critical_point_limit():
    """Close to T_c = 1 the two branches merge at rho_c = 1 like sqrt(1 - T):
    (rho_L - rho_V) / 2 -> 2 sqrt(1 - T) for the van der Waals fluid."""
    for eps in (1e-3, 1e-4):
        rv, rl = thermo.maxwell(1.0 - eps)
        assert 0.5 * (rl - rv) == pytest.approx(2.0 * math.sqrt(eps), rel=3 * math.sqrt(eps))


def test_surface_tension_closed_form_equals_profile_integral():
    """sigma = int sqrt(2 kappa W) d rho (closed form) equals kappa int rho'^2 dx
    on the relaxed flat profile, which solves kappa rho'^2 = 2 W(rho); the
    profile is built here by integrating that ODE."""
    T, kappa = 0.8, 1e-4
    rv, rl = thermo.maxwell(T)
    mid = 0.5 * (rv + rl)
    drho = lambda x, r: [math.sqrt(max(2.0 * thermo.grand_potential_excess(r[0], T) / kappa, 0.0))]
    xs = np.linspace(0.0, 0.25, 50001)
    up = integrate.solve_ivp(drho, (0.0, xs[-1]), [mid], t_eval=xs, rtol=1e-11, atol=1e-13)
    down = integrate.solve_ivp(lambda x, r: [-v for v in drho(x, r)], (0.0, xs[-1]), [mid], t_eval=xs,
                               rtol=1e-11, atol=1e-13)
    prof = np.concatenate([down.y[0][::-1], up.y[0][1:]])
    assert prof[0] - rv < 1e-5 and rl - prof[-1] < 1e-5
    dx = xs[1] - xs[0]
    s_prof = kappa * np.sum(np.gradient(prof, dx) ** 2) * dx
    s_closed = thermo.surface_tension(T, kappa)
    assert s_prof == pytest.approx(s_closed, rel=2e-4)


def test_surface_tension_against_printed_lattice_value():
    """Sec. III A prints sigma = 4.8747e-3 (ds = 1/256) and 4.8754e-3 (ds = 1/128)
    from relaxed lattice profiles at T = 0.8, kappa = 1e-4; the continuum value
    lies 0.3% above them."""
    s = thermo.surface_tension(0.8, 1e-4)
    for key in ("ds_1_256", "ds_1_128"):
        printed = PAPER["surface_tension_T0.8_kappa1e-4"][key]
        assert s == pytest.approx(printed, rel=5e-3)
        assert s > printed


def test_critical_radius_against_printed_value():
    """Eq. (raggio_c) at T = 0.8, rho_ext = 1.923 with the printed sigma gives
    75.5 ds (ds = 1/256); Sec. III B finds 76.5 ds in the lattice runs, a
    slight overestimation at the larger rho_ext."""
    g = PAPER["critical_radius"]
    sigma = PAPER["surface_tension_T0.8_kappa1e-4"]["ds_1_256"]
    rc = thermo.critical_radius(0.8, g["rho_ext"], sigma) / g["ds"]
    assert rc == pytest.approx(75.5, abs=0.1)
    assert 0.97 * g["R_c_over_ds"] < rc < g["R_c_over_ds"]


def test_critical_radius_ignores_linear_terms_in_psi():
    """The paper's free energy rho T ln(3 rho/(3 - rho)) - 9/8 rho^2 differs from
    the general-(a, b) form by a term linear in rho, to which Eq. (raggio_c) is
    blind (the bracket weights sum to zero on linear functions)."""
    T, rho_ext, sigma = 0.8, 1.9, 4.8747e-3
    rv, rl = thermo.maxwell(T)
    psi_paper = lambda r: r * T * math.log(3.0 * r / (3.0 - r)) - 9.0 / 8.0 * r * r
    brace = (psi_paper(rv) - psi_paper(rho_ext)) + (rho_ext - rv) / (rl - rho_ext) * (psi_paper(rl) - psi_paper(rho_ext))
    assert -0.5 * sigma / brace == pytest.approx(thermo.critical_radius(T, rho_ext, sigma), rel=1e-12)


@pytest.mark.parametrize("sigma,mu", [(0.0, 0.0), (0.01, 0.0), (0.01, 0.02)])
def test_rayleigh_plesset_energy_balance(sigma, mu):
    """For r_inf >> R, Eq. (eq:rp) is the energy balance of the 2D potential
    flow: with constant dp, E = R^2 R'^2 ln(r_inf/R) - (dp/rho) R^2 + 2 sigma R / rho
    obeys dE/dt = -4 mu R'^2 / rho.  The RK4 solution must keep that budget."""
    rho, dp, r_inf = 1.5, 0.02, 1e8
    t, R, V = thermo.rayleigh_plesset_rk4(1.0, 0.01, 0.0, 20.0, 20000, rho, mu, sigma, r_inf, lambda tt: dp)
    E = R * R * V * V * np.log(r_inf / R) - dp / rho * R * R + 2.0 * sigma * R / rho
    diss = integrate.cumulative_trapezoid(4.0 * mu * V * V / rho, t, initial=0.0)
    np.testing.assert_allclose(E + diss, E[0], rtol=0, atol=1e-7 * np.abs(E).max())
    assert R[-1] > R[0]
