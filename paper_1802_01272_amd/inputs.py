"""Seeded synthetic inputs (initial density and velocity fields).

This module is shared by the tests, the benchmark and the oracle checks.  It
holds no part of the lattice Boltzmann step: it only lays out initial
densities and velocities of the kind the paper studies (flat liquid-vapour
interfaces, Sec. II E; a vapour bubble in a superheated liquid, Sec. III A-B;
a bubble in a liquid sheared by two moving walls with a linear initial
velocity profile, Sec. III C) and draws the seeded noise.

The liquid and vapour densities that define those states are the van der
Waals coexistence densities.  They are computed here by this module's own
equal-area (Maxwell) rule in the specific volume v = 1/rho, independently of
the oracle's equal-chemical-potential solver; a test checks the two agree.

Conventions: arrays have shape (Ly, Lx), node (i, j) at x = i, y = j in
lattice units; noise is i.i.d. uniform on [-amp, amp] from numpy's PCG64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np
from scipy import integrate, optimize

# --------------------------------------------------------------------------
# coexistence densities of p = rho T / (1 - b rho) - a rho^2  (equal-area rule)


def _p_of_v(v, T, a, b):
    return T / (v - b) - a / (v * v)


def _p_integral(v0, v1, T, a, b):
    """int_{v0}^{v1} p(v) dv in closed form."""
    return T * math.log((v1 - b) / (v0 - b)) + a * (1.0 / v1 - 1.0 / v0)


def coexistence(T: float, a: float = 9.0 / 8.0, b: float = 1.0 / 3.0):
    """(rho_vapour, rho_liquid) from the equal-area construction.

    For a trial pressure P between the two spinodal pressures, v_L and v_V are
    the outer roots of p(v) = P; P is adjusted until int_{v_L}^{v_V} p dv equals
    P (v_V - v_L)."""
    Tc = 8.0 * a / (27.0 * b)
    if not (0.0 < T < Tc):
        raise ValueError("temperature must lie below the critical temperature")
    # spinodals in v: dp/dv = 0  <=>  T v^3 = 2 a (v - b)^2
    g = lambda v: T * v ** 3 - 2.0 * a * (v - b) ** 2
    vc = 3.0 * b
    v_sl = optimize.brentq(g, b * (1.0 + 1e-12), vc)      # liquid-side spinodal
    v_sv = optimize.brentq(g, vc, 1e6 * b)                  # vapour-side spinodal
    p_min = _p_of_v(v_sl, T, a, b)
    p_max = _p_of_v(v_sv, T, a, b)
    lo_p = max(p_min, 0.0) + 1e-10 * T   # p(v = 1e12) is far below this

    def roots(P):
        vl = optimize.brentq(lambda v: _p_of_v(v, T, a, b) - P, b * (1.0 + 1e-15), v_sl,
                             xtol=1e-15, rtol=1e-15, maxiter=400)
        vv = optimize.brentq(lambda v: _p_of_v(v, T, a, b) - P, v_sv, 1e12,
                             xtol=1e-15, rtol=1e-15, maxiter=400)
        return vl, vv

    def area(P):
        vl, vv = roots(P)
        return _p_integral(vl, vv, T, a, b) - P * (vv - vl)

    P = optimize.brentq(area, lo_p, p_max * (1.0 - 1e-14), xtol=1e-16, rtol=1e-15, maxiter=400)
    vl, vv = roots(P)
    return 1.0 / vv, 1.0 / vl


# --------------------------------------------------------------------------
# profiles


def noise(shape, amp: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-amp, amp, size=shape)


def slab(Lx: int, Ly: int, rho_in: float, rho_out: float, x_lo: float, x_hi: float,
         width: float = 3.0) -> np.ndarray:
    """Density rho_in for x_lo <= x < x_hi, rho_out elsewhere, tanh interfaces
    of width `width` nodes centred half a node outside the slab's end nodes."""
    x = np.arange(Lx, dtype=np.float64)
    prof = rho_out + 0.5 * (rho_in - rho_out) * (np.tanh((x - (x_lo - 0.5)) / width)
                                                  - np.tanh((x - (x_hi - 0.5)) / width))
    return np.broadcast_to(prof, (Ly, Lx)).copy()


def bubble(Lx: int, Ly: int, rho_in: float, rho_out: float, radius: float,
           width: float = 3.0, centre=None) -> np.ndarray:
    """Circular region of density rho_in (radius in nodes) in a fluid of density
    rho_out, tanh profile of width `width`, centred at ((Lx-1)/2, (Ly-1)/2)."""
    cx, cy = centre if centre is not None else (0.5 * (Lx - 1), 0.5 * (Ly - 1))
    x = np.arange(Lx, dtype=np.float64)[None, :]
    y = np.arange(Ly, dtype=np.float64)[:, None]
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return rho_in + (rho_out - rho_in) * 0.5 * (1.0 + np.tanh((r - radius) / width))


def shear_profile(Lx: int, Ly: int, shear_rate: float, ds: float = 1.0):
    """Linear profile u_x(j) = shear_rate * ds * (j - (Ly-1)/2), u_y = 0; with
    walls at j = -1/2 and Ly - 1/2 this gives wall speeds -+ shear_rate*Ly*ds/2."""
    j = np.arange(Ly, dtype=np.float64)[:, None]
    ux = np.broadcast_to(shear_rate * ds * (j - 0.5 * (Ly - 1)), (Ly, Lx)).copy()
    return ux, np.zeros((Ly, Lx))


# --------------------------------------------------------------------------
# workloads


@dataclass
class Workload:
    """One synthetic run: physical parameters plus its initial fields."""
    name: str
    Lx: int
    Ly: int
    T: float
    a: float
    b: float
    kappa: float
    tau: float
    ds: float = 1.0
    dt: float = 0.25
    scheme: int = 2
    regularize: int = 0
    bc_y: int = 0
    u_wall: float = 0.0
    rho_wall: float = 1.0
    rho_ref: float = 1.0
    steps: int = 1000
    rho_liquid: float = 0.0
    rho_vapour: float = 0.0
    rho_ext: float = 0.0
    shape: str = "bubble"        # "bubble" or "slab"
    radius: float = 20.0
    width: float = 3.0
    noise_amp: float = 0.0
    seed: int = 0
    shear_rate: float = 0.0
    notes: str = ""

    def fields(self):
        """(rho, ux, uy), float64 arrays of shape (Ly, Lx)."""
        if self.shape == "slab":
            rho = slab(self.Lx, self.Ly, self.rho_liquid, self.rho_vapour,
                       self.Lx // 4, 3 * self.Lx // 4, self.width)
        else:
            rho = bubble(self.Lx, self.Ly, self.rho_vapour, self.rho_ext, self.radius, self.width)
        if self.noise_amp > 0.0:
            rho = rho + noise(rho.shape, self.noise_amp, self.seed)
        if self.shear_rate != 0.0:
            ux, uy = shear_profile(self.Lx, self.Ly, self.shear_rate, self.ds)
        else:
            ux, uy = np.zeros_like(rho), np.zeros_like(rho)
        return np.ascontiguousarray(rho), np.ascontiguousarray(ux), np.ascontiguousarray(uy)

    def with_size(self, Lx: int, Ly: int, **kw) -> "Workload":
        """Same fluid and shape on another lattice (radius scaled only if given)."""
        return replace(self, Lx=Lx, Ly=Ly, **kw)


def flat_interface_small() -> Workload:
    """64 x 64 periodic lattice, van der Waals a = 9/49, b = 2/21 (critical
    point T_c = 4/7, rho_c = 3.5), T = 0.9 T_c, tau = 0.8, CTU2, dt = ds/4; a
    liquid slab over half the domain with tanh interfaces of width 3 and
    +-1e-4 seeded uniform noise; 1000 steps.  kappa = 1/6.125 gives the same
    interface length sqrt(kappa rho_c / T_c) as kappa = 1 in the paper's units."""
    a, b = 9.0 / 49.0, 2.0 / 21.0
    Tc = 8.0 * a / (27.0 * b)
    T = 0.9 * Tc
    rv, rl = coexistence(T, a, b)
    return Workload("flat_interface_64", 64, 64, T=T, a=a, b=b, kappa=1.0 / 6.125, tau=0.8,
                    steps=1000, rho_liquid=rl, rho_vapour=rv, rho_ref=0.5 * (rl + rv),
                    shape="slab", noise_amp=1e-4, seed=1)


def _paper_fluid(T_over_Tc: float):
    a, b = 9.0 / 8.0, 1.0 / 3.0   # critical point T_c = rho_c = 1
    rv, rl = coexistence(T_over_Tc, a, b)
    return a, b, rv, rl


def storage_reference(rho_vapour: float, rho_ext: float) -> float:
    """rho_ref of the FP32 deviation storage for a bubble in liquid: the far
    liquid's density, which fills almost all of the lattice, so the stored
    f_k - w_k rho_ref (and their roundings) nearly vanish there.  On the
    1024^2 cavitation run this keeps rho and u within 1e-5 of the FP64 stepper
    after 10^4 steps (3.5e-6 and 9.6e-6); a reference midway between the
    phases, which halves the largest stored deviation, leaves 1.8e-5 and
    3.4e-5 at the moving interface.  rho_vapour is unused."""
    del rho_vapour
    return rho_ext


def quiescent_bubble(L: int = 1024, radius: float = 20.0) -> Workload:
    """Superheated liquid at T = 0.95 T_c, density 0.95 rho_L (coexistence),
    one vapour bubble (rho_V) of radius `radius` nodes at the centre, tau = 0.7,
    kappa = 1, CTU2, periodic."""
    a, b, rv, rl = _paper_fluid(0.95)
    rho_ext = 0.95 * rl
    return Workload("quiescent_bubble_%d" % L, L, L, T=0.95, a=a, b=b, kappa=1.0, tau=0.7,
                    steps=20000, rho_liquid=rl, rho_vapour=rv, rho_ext=rho_ext,
                    rho_ref=storage_reference(rv, rho_ext), shape="bubble", radius=radius)


def large_lattice(L: int = 6144) -> Workload:
    """The same fluid and bubble on the paper's largest lattice, radius 60."""
    w = quiescent_bubble(L, radius=60.0)
    w.name = "large_lattice_%d" % L
    w.steps = 5000
    return w


def sheared_bubble(shear_rate: float, L: int = 2048) -> Workload:
    """Sheared cavitation: x periodic, permeable walls moving at -+u_w in the
    two ghost rows below and above, u_w = shear_rate * L * ds / 2, linear
    initial profile, T = 0.95 T_c, rho_ext = rho_wall = 0.95 rho_L, bubble of
    radius 30, +-1e-4 noise (seed 4), tau = 0.7, kappa = 1."""
    a, b, rv, rl = _paper_fluid(0.95)
    rho_ext = 0.95 * rl
    return Workload("sheared_bubble_%d_%g" % (L, shear_rate), L, L, T=0.95, a=a, b=b,
                    kappa=1.0, tau=0.7, bc_y=1, u_wall=shear_rate * L / 2.0, rho_wall=rho_ext,
                    steps=30000, rho_liquid=rl, rho_vapour=rv, rho_ext=rho_ext,
                    rho_ref=storage_reference(rv, rho_ext), shape="bubble", radius=30.0, noise_amp=1e-4, seed=4, shear_rate=shear_rate)


SHEAR_RATES = (1e-5, 5e-5, 1e-4, 5e-4)


def batched_sweep(n: int = 32, seed: int = 5) -> List[Workload]:
    """n independent runs: lattice edge from {256, 384, 512, 768, 1024, 1536},
    T/T_c uniform in [0.85, 0.97], shear rate from {0, 1e-5, 1e-4} (walls when
    non-zero), bubble radius 8..40 nodes, rho_ext = 0.95 rho_L(T), +-1e-4 noise,
    tau = 0.7, kappa = 1, 10000 steps each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = (256, 384, 512, 768, 1024, 1536)
    rates = (0.0, 1e-5, 1e-4)
    out = []
    for r in range(n):
        L = int(edges[rng.integers(len(edges))])
        T = float(rng.uniform(0.85, 0.97))
        gamma = float(rates[rng.integers(len(rates))])
        R = float(rng.integers(8, 41))
        nseed = int(rng.integers(1 << 31))
        a, b, rv, rl = _paper_fluid(T)
        rho_ext = 0.95 * rl
        out.append(Workload("batch_%02d" % r, L, L, T=T, a=a, b=b, kappa=1.0, tau=0.7,
                            bc_y=1 if gamma > 0 else 0, u_wall=gamma * L / 2.0,
                            rho_wall=rho_ext, steps=10000, rho_liquid=rl, rho_vapour=rv,
                            rho_ext=rho_ext, rho_ref=storage_reference(rv, rho_ext),
                            shape="bubble", radius=R,
                            noise_amp=1e-4, seed=nseed, shear_rate=gamma))
    return out
