"""Closed forms of the van der Waals fluid -- TEST INFRASTRUCTURE ONLY.

Used by the tests to pin the oracle (and, through it, the HIP path) to the
paper's physics:

* the van der Waals pressure, Eq. (evdw), and bulk free energy, Eq. (free-en2),
  written for general constants (a, b) (the paper: a = 9/8, b = 1/3);
* the Maxwell construction for the coexistence densities (Sec. II E);
* the flat-interface surface tension sigma = kappa * int (d rho/dx)^2 dx, which
  follows from the pressure tensor, Eq. (pr-tensor), and its closed form
  sigma = int_{rho_V}^{rho_L} sqrt(2 kappa W(rho)) d rho with the excess
  grand-potential density W = psi - mu_coex rho + p_coex;
* the critical radius, Eq. (eq:raggio_c);
* the two-dimensional Rayleigh-Plesset equation, Eq. (eq:rp), integrated with
  the classical fourth-order Runge-Kutta method.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

PAPER_A = 9.0 / 8.0
PAPER_B = 1.0 / 3.0


def pressure(rho, T, a=PAPER_A, b=PAPER_B):
    """Eq. (evdw): p = rho T / (1 - b rho) - a rho^2."""
    return rho * T / (1.0 - b * rho) - a * rho * rho


def free_energy(rho, T, a=PAPER_A, b=PAPER_B):
    """Eq. (free-en2) for general (a, b): psi = rho T ln(rho / (1 - b rho)) - a rho^2.

    With a = 9/8, b = 1/3 this is rho T ln(3 rho / (3 - rho)) - 9/8 rho^2; the
    paper's form differs from this one only by a term linear in rho (T ln 3 rho
    for b = 1/3), which changes neither pressure differences nor Eq. (raggio_c).
    """
    return rho * T * np.log(rho / (1.0 - b * rho)) - a * rho * rho


def chemical_potential(rho, T, a=PAPER_A, b=PAPER_B):
    """mu = d psi / d rho."""
    return T * np.log(rho / (1.0 - b * rho)) + T / (1.0 - b * rho) - 2.0 * a * rho


def spinodals(T, a=PAPER_A, b=PAPER_B):
    """Densities where dp/drho = 0 (vapour side, liquid side)."""
    dp = lambda r: T / (1.0 - b * r) ** 2 - 2.0 * a * r
    rc = 1.0 / (3.0 * b)
    lo = optimize.brentq(dp, 1e-9, rc)
    hi = optimize.brentq(dp, rc, (1.0 - 1e-9) / b)
    return lo, hi


def maxwell(T, a=PAPER_A, b=PAPER_B):
    """Coexistence densities (rho_V, rho_L): equal pressure and equal chemical
    potential.  Bracketed: for a trial pressure P between the spinodal
    pressures, the vapour and liquid branches each have one root of p = P, and
    mu(vapour) - mu(liquid) changes sign once over that pressure interval."""
    sv, sl = spinodals(T, a, b)
    p_lo = max(pressure(sl, T, a, b), 0.0) * (1.0 + 1e-12) + 1e-300
    p_hi = pressure(sv, T, a, b) * (1.0 - 1e-12)

    def branches(P):
        rv = optimize.brentq(lambda r: pressure(r, T, a, b) - P, 1e-300, sv, xtol=1e-300, rtol=1e-15, maxiter=500)
        rl = optimize.brentq(lambda r: pressure(r, T, a, b) - P, sl, (1.0 - 1e-15) / b, xtol=1e-300, rtol=1e-15, maxiter=500)
        return rv, rl

    def gap(P):
        rv, rl = branches(P)
        return chemical_potential(rv, T, a, b) - chemical_potential(rl, T, a, b)

    P = optimize.brentq(gap, p_lo, p_hi, xtol=1e-300, rtol=1e-15, maxiter=500)
    rv, rl = branches(P)
    return float(rv), float(rl)


def grand_potential_excess(rho, T, a=PAPER_A, b=PAPER_B):
    """W(rho) = psi - mu_coex rho + p_coex, >= 0 between the binodals."""
    rv, rl = maxwell(T, a, b)
    mu = chemical_potential(rv, T, a, b)
    p = pressure(rv, T, a, b)
    return free_energy(rho, T, a, b) - mu * rho + p


def surface_tension(T, kappa, a=PAPER_A, b=PAPER_B):
    """sigma = int_{rho_V}^{rho_L} sqrt(2 kappa W(rho)) d rho (flat interface)."""
    rv, rl = maxwell(T, a, b)
    f = lambda r: math.sqrt(max(2.0 * kappa * grand_potential_excess(r, T, a, b), 0.0))
    val, _ = integrate.quad(f, rv, rl, limit=200, epsabs=1e-14, epsrel=1e-12)
    return val


def surface_tension_from_profile(rho, ds, kappa):
    """sigma = kappa int (d rho/dx)^2 dx along a 1D profile (centred differences,
    periodic), the tension that follows from Eq. (pr-tensor)."""
    rho = np.asarray(rho, dtype=np.float64)
    d = (np.roll(rho, -1) - np.roll(rho, 1)) / (2.0 * ds)
    return kappa * float(np.sum(d * d) * ds)


def critical_radius(T, rho_ext, sigma, a=PAPER_A, b=PAPER_B):
    """Eq. (eq:raggio_c): bubble radius that neither grows nor shrinks."""
    rv, rl = maxwell(T, a, b)
    psi = lambda r: float(free_energy(r, T, a, b))
    brace = (psi(rv) - psi(rho_ext)) + (rho_ext - rv) / (rl - rho_ext) * (psi(rl) - psi(rho_ext))
    return -0.5 * sigma / brace


def rayleigh_plesset_rhs(t, state, rho_L, mu_L, sigma, r_inf, dp_of_t):
    """Eq. (eq:rp) solved for d^2R/dt^2.  state = (R, dR/dt);
    dp_of_t(t) = p_B(t) - p_inf(t)."""
    R, V = state
    lg = math.log(r_inf / R)
    rhs = (dp_of_t(t) / rho_L - sigma / (rho_L * R) - 2.0 * mu_L * V / (rho_L * R)
           + 0.5 * (1.0 - R * R / (r_inf * r_inf)) * V * V)
    Rdd = (rhs / lg - V * V) / R
    return np.array([V, Rdd])


def rayleigh_plesset_rk4(R0, V0, t0, t1, nsteps, rho_L, mu_L, sigma, r_inf, dp_of_t):
    """Integrate Eq. (eq:rp) from t0 to t1 with classical RK4; returns (t, R, V)."""
    h = (t1 - t0) / nsteps
    ts = np.empty(nsteps + 1)
    ys = np.empty((nsteps + 1, 2))
    y = np.array([R0, V0], dtype=np.float64)
    t = t0
    ts[0], ys[0] = t, y
    f = lambda tt, yy: rayleigh_plesset_rhs(tt, yy, rho_L, mu_L, sigma, r_inf, dp_of_t)
    for n in range(nsteps):
        k1 = f(t, y)
        k2 = f(t + h / 2, y + h / 2 * k1)
        k3 = f(t + h / 2, y + h / 2 * k2)
        k4 = f(t + h, y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        t = t0 + (n + 1) * h
        ts[n + 1], ys[n + 1] = t, y
    return ts, ys[:, 0], ys[:, 1]


def taylor_deformation_slope(lam):
    """Small-Ca Taylor law D = (19 lam + 16)/(16 lam + 16) Ca; returns the slope."""
    return (19.0 * lam + 16.0) / (16.0 * lam + 16.0)
