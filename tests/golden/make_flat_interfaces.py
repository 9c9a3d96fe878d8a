"""Writes the relaxed flat-interface density profiles that
tests/test_physics_pins.py starts from.  Calls only the CPU oracle.

The parameters are those of Sec. III A (T = 0.8) and of the phase diagram of
Sec. II E (T = 0.7, 0.6): CTU2, tau = 1e-3, dt = 1e-4, ds = 1/256, kappa =
1e-4, van der Waals fluid a = 9/8, b = 1/3.  The lattice is one column wide
and 256 rows high (periodic), a liquid slab over rows 64..191 between two
vapour layers; it starts from tanh profiles at the Maxwell densities and is
advanced `--steps` steps (a few minutes per temperature).  The profile rho(j)
is written to flat_interface_T<T>.txt, one value per line.

Usage: python tests/golden/make_flat_interfaces.py [--steps 600000] [T ...]
"""
import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as o  # noqa: E402
from oracle import thermo  # noqa: E402

N, DS, DT, TAU, KAPPA = 256, 1.0 / 256, 1e-4, 1e-3, 1e-4


def params(T):
    return o.Params(Lx=1, Ly=N, ds=DS, dt=DT, tau=TAU, T=T, kappa=KAPPA, scheme=2)


def initial_profile(T):
    rv, rl = thermo.maxwell(T)
    j = np.arange(N)
    d = np.minimum(np.abs(j - N / 4), np.abs(j - 3 * N / 4))
    s = np.where((j >= N / 4) & (j < 3 * N / 4), 1.0, -1.0)
    return 0.5 * (rl + rv) + 0.5 * (rl - rv) * np.tanh(s * d / 4.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=600000)
    ap.add_argument("T", nargs="*", type=float, default=[0.8, 0.7, 0.6])
    args = ap.parse_args()
    o.set_num_threads(1)
    for T in args.T:
        p = params(T)
        z = np.zeros((N, 1))
        f = o.init(p, initial_profile(T).reshape(N, 1), z, z)
        f = o.run(p, f, args.steps)
        rho = f.sum(axis=0)[:, 0]
        path = os.path.join(HERE, "flat_interface_T%.1f.txt" % T)
        with open(path, "w") as fh:
            fh.write("# relaxed flat interface, oracle, CTU2, T=%.2f tau=%g dt=%g ds=1/256 kappa=%g, "
                     "%d steps from tanh profiles at the Maxwell densities\n" % (T, TAU, DT, KAPPA, args.steps))
            fh.write("# written by tests/golden/make_flat_interfaces.py; rho(j), j = 0..%d\n" % (N - 1))
            for v in rho:
                fh.write("%.17g\n" % v)
        print("wrote", path, "rho_V %.6f rho_L %.6f" % (rho[0], rho[N // 2]), flush=True)


if __name__ == "__main__":
    main()
