"""Shared helpers of the GPU tests: seeded states and oracle parameter mapping."""
import numpy as np

import oracle as o
from paper_1802_01272_amd import lbm


def oracle_params(p: "lbm.Params") -> o.Params:
    return o.Params(Lx=p.Lx, Ly=p.Ly, ds=p.ds, dt=p.dt, tau=p.tau, T=p.T, a=p.a, b=p.b, kappa=p.kappa,
                    scheme=p.scheme, regularize=p.regularize, bc_y=p.bc_y, u_wall=p.u_wall,
                    rho_wall=p.rho_wall, clamp_radius=p.clamp_radius, clamp_rho=p.clamp_rho)


def random_state(p: "lbm.Params", seed: int, amp: float = 0.03, rho_mean: float = 1.2, rho_amp: float = 0.15):
    """f = f^eq(rho, u) * (1 + amp * noise): a non-equilibrium state with O(amp)
    departures in every Hermite order, drawn with numpy's PCG64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = rho_mean + rho_amp * rng.uniform(-1, 1, (p.Ly, p.Lx))
    ux = 0.05 * rng.standard_normal((p.Ly, p.Lx))
    uy = 0.05 * rng.standard_normal((p.Ly, p.Lx))
    f = o.init(oracle_params(p), rho, ux, uy)
    return np.ascontiguousarray(f * (1.0 + amp * rng.standard_normal(f.shape)))


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def field_errors(rho, ux, uy, rho_ref, ux_ref, uy_ref):
    """Pointwise relative density error and velocity error normalised by the
    largest reference speed (u -> 0 in the bulk)."""
    umax = max(np.max(np.hypot(ux_ref, uy_ref)), 1e-300)
    du = np.hypot(ux - ux_ref, uy - uy_ref)
    drho = np.abs(rho - rho_ref) / np.abs(rho_ref)
    return {
        "rho_max": float(drho.max()), "rho_rms": float(np.sqrt(np.mean(drho ** 2))),
        "u_max": float(du.max() / umax), "u_rms": float(np.sqrt(np.mean(du ** 2)) / umax),
    }
