"""The oracle's whole step against the flat-interface values the paper prints.

Sec. III A prints the surface tension of a relaxed flat interface (T = 0.8,
kappa = 1e-4, tau = 1e-3, dt = 1e-4, ds = 1/256, CTU2): sigma = 4.8747e-3,
and the coexistence densities rho_V = 0.23967, rho_L = 1.9327 that the
simulations start from.  Sec. II E states that the planar interface's
densities agree with the Maxwell construction for T >= 0.70 and that the
vapour density falls about 8% below it at T = 0.60, with the same numerics.

Each test restarts the oracle from a relaxed profile written by
tests/golden/make_flat_interfaces.py (oracle only; f = f^eq(rho, 0) from the
stored density), lets the restart's acoustic transient pass, and reads the
plateau densities and sigma = kappa int (d rho/dy)^2 dy across one interface,
averaged over a few samples.  A stencil or force slip moves these within the
run: the second-order 24-neighbour gradient, for example, leaves sigma 1.9%
low and the vapour 5% low at T = 0.8 (15% at 0.7, 44% at 0.6).
"""
import json
import os

import numpy as np
import pytest

import oracle as o
from oracle import thermo

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "paper_values.json")) as fh:
    PAPER = json.load(fh)

pytestmark = pytest.mark.slow

N, DS, DT, TAU, KAPPA = 256, 1.0 / 256, 1e-4, 1e-3, 1e-4


def relaxed_interface(T, settle=8000, samples=8, every=500):
    rho0 = np.loadtxt(os.path.join(HERE, "golden", "flat_interface_T%.1f.txt" % T))
    assert rho0.shape == (N,)
    p = o.Params(Lx=1, Ly=N, ds=DS, dt=DT, tau=TAU, T=T, kappa=KAPPA, scheme=2)
    z = np.zeros((N, 1))
    f = o.run(p, o.init(p, rho0.reshape(N, 1), z, z), settle)
    acc = []
    for _ in range(samples):
        f = o.run(p, f, every)
        rho = f.sum(axis=0)[:, 0]
        drho = (np.roll(rho, -1) - np.roll(rho, 1)) / (2 * DS)
        acc.append((rho[0], rho[N // 2], KAPPA * np.sum(drho[:N // 2] ** 2) * DS))
    return np.mean(acc, axis=0)


def test_flat_interface_surface_tension_and_densities_at_T08():
    rv, rl, sigma = relaxed_interface(0.8)
    printed = PAPER["surface_tension_T0.8_kappa1e-4"]["ds_1_256"]
    assert sigma == pytest.approx(printed, rel=3e-3)
    co = PAPER["coexistence_T0.8"]
    assert rl == pytest.approx(co["rho_L"], rel=1e-3)
    assert rv == pytest.approx(co["rho_V_more_digits"], rel=0.015)


@pytest.mark.parametrize("T", [0.7, 0.6])
def test_phase_diagram_vapour_branch(T):
    """T = 0.7: within a few percent of Maxwell (the paper's agreement);
    T = 0.6: the vapour falls clearly below it, by about the printed 8%."""
    rv, rl, _ = relaxed_interface(T)
    mv, ml = thermo.maxwell(T)
    assert rl == pytest.approx(ml, rel=1e-3)
    dev = 1.0 - rv / mv
    if T >= PAPER["phase_diagram"]["agreement_from_T"]:
        assert 0.0 <= dev < 0.04
    else:
        assert 0.5 * PAPER["phase_diagram"]["vapour_deviation_T0.6"] < dev < 1.5 * PAPER["phase_diagram"]["vapour_deviation_T0.6"]
