"""The seeded input generators: coexistence densities and workload layout."""
import numpy as np
import pytest

from oracle import thermo
from paper_1802_01272_amd import inputs as I


@pytest.mark.parametrize("T", [0.6, 0.7, 0.8, 0.85, 0.9, 0.95, 0.97])
def test_input_coexistence_agrees_with_oracle_maxwell(T):
    rv, rl = I.coexistence(T)
    ov, ol = thermo.maxwell(T)
    assert rv == pytest.approx(ov, rel=1e-10)
    assert rl == pytest.approx(ol, rel=1e-10)


def test_general_constants_coexistence():
    a, b = 9 / 49, 2 / 21
    rv, rl = I.coexistence(0.9 * 4 / 7, a, b)
    ov, ol = thermo.maxwell(0.9 * 4 / 7, a, b)
    assert rv == pytest.approx(ov, rel=1e-10) and rl == pytest.approx(ol, rel=1e-10)
    # same reduced state as the paper's units, rescaled by rho_c = 3.5
    pv, pl = I.coexistence(0.9)
    assert rv == pytest.approx(3.5 * pv, rel=1e-10) and rl == pytest.approx(3.5 * pl, rel=1e-10)


def test_noise_is_seeded_and_bounded():
    a = I.noise((5, 7), 1e-4, 3)
    b = I.noise((5, 7), 1e-4, 3)
    assert np.array_equal(a, b)
    assert np.abs(a).max() <= 1e-4
    assert not np.array_equal(a, I.noise((5, 7), 1e-4, 4))


def test_workload_fields():
    w = I.quiescent_bubble(64, radius=10)
    rho, ux, uy = w.fields()
    assert rho.shape == (64, 64) and not ux.any() and not uy.any()
    assert rho.min() == pytest.approx(w.rho_vapour, abs=3e-3)
    assert rho[0, 0] == pytest.approx(w.rho_ext, abs=1e-6)
    assert w.rho_ext == pytest.approx(0.95 * 1.461727, abs=1e-6)
    s = I.sheared_bubble(1e-4, L=32)
    _, ux, _ = s.fields()
    assert s.u_wall == pytest.approx(1e-4 * 16)
    np.testing.assert_allclose(ux[:, 0], 1e-4 * (np.arange(32) - 15.5))
    f = I.flat_interface_small()
    rho, _, _ = f.fields()
    assert rho[:, 32].mean() == pytest.approx(f.rho_liquid, rel=1e-3)
    assert rho[:, 0].mean() == pytest.approx(f.rho_vapour, rel=1e-2)


def test_batched_sweep_draw():
    ws = I.batched_sweep()
    assert len(ws) == 32
    assert all(w.Lx in (256, 384, 512, 768, 1024, 1536) for w in ws)
    assert all(0.85 <= w.T <= 0.97 for w in ws)
    assert all(8 <= w.radius <= 40 for w in ws)
    assert all((w.bc_y == 1) == (w.shear_rate > 0) for w in ws)
    assert [w.Lx for w in ws] == [w.Lx for w in I.batched_sweep()]
