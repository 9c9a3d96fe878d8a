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


def box_rows(box, Ly, walls):
    """Rows [r0, r1) of the cut for box (j0, j1, i0, i1): four rows of margin
    (the reach of one step), wrapped periodically, or clipped at the walls."""
    j0, j1 = box[0], box[1]
    if walls:
        r0, r1 = max(j0 - 4, 0), min(j1 + 4, Ly)
        assert (r0 == 0 or r0 == j0 - 4) and (r1 == Ly or r1 == j1 + 4)
        return r0, r1
    return j0 - 4, j1 + 4


def oracle_box_step(op, fcut, box, r0, Ly, walls):
    """The oracle's step of box (j0, j1, i0, i1) from a cut of the input state
    (rows [r0, r0 + fcut.shape[1]), columns [i0 - 4, i1 + 4), wrapped): the cut
    is stepped as a small lattice, periodic, or with walls when it reaches a
    wall row (its own wall on the far side lies out of the step's reach)."""
    j0, j1, i0, i1 = box
    q = o.Params(**{k: getattr(op, k) for k in op.__dataclass_fields__})
    q.Lx, q.Ly = fcut.shape[2], fcut.shape[1]
    q.bc_y = 1 if walls and (r0 == 0 or r0 + fcut.shape[1] == Ly) else 0
    return o.step_region(q, np.ascontiguousarray(fcut), 4, 4 + (i1 - i0), j0 - r0, j1 - r0)
