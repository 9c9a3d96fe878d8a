"""Parity of the HIP stepper (through the C ABI) with the FP64 CPU oracle.

Tolerances, derived from the arithmetic (every kernel sums in a different
order than the oracle and contracts multiply-adds):
  * FP64 storage: one step agrees to some tens of units in the last place of
    the largest f (bound 2e-14 relative, about 90 ulps: the force divides by
    rho and 1 - b rho and differences the van der Waals pressure over the
    stencils); after many steps rounding differences stay below 1e-10
    relative in rho and u.
  * FP32 deviation storage: the oracle steps the GPU's own stored input, so
    one step differs by the rounding of the new deviation to FP32 (stochastic:
    under one ulp, at most 2^-23 of the value) plus the FP32 arithmetic of
    the CTU2 corrections (a few ulps of increments below a tenth of f): bound
    3e-7 of max|f|; rho and u after many steps follow the 1e-5 bar (u
    normalised by its largest value).
"""
import numpy as np
import pytest

import oracle as o
from gpu_helpers import box_rows, field_errors, oracle_box_step, oracle_params, random_state, rel_err
from paper_1802_01272_amd import inputs as I

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_1802_01272_amd.lbm")

F64_STEP = 2e-14
F32_STEP = 3e-7


def make_params(Lx, Ly, scheme=2, reg=0, bc=0, precision=0, **kw):
    p = lbm.Params(Lx=Lx, Ly=Ly, T=0.93, kappa=0.8, tau=0.7, scheme=scheme, regularize=reg, bc_y=bc,
                   u_wall=0.04 if bc else 0.0, rho_wall=1.25, precision=precision, rho_ref=1.2)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def gpu_step_from(p, f, nsteps=1, launch=None, start_step=0):
    """f advanced by nsteps single-run steps, starting at step count
    start_step (FP32 storage: the stochastic rounding follows the step
    count)."""
    run = lbm.Run(p, 1.0, 0.0, 0.0)
    if launch:
        run.set_launch(*launch)
    run.step(start_step)
    run.set_f(f)
    run.step(nsteps)
    out = run.get_f()
    run.close()
    return out


# ---------------------------------------------------------------- init / I-O

@pytest.mark.parametrize("precision", [0, 1])
def test_init_is_equilibrium(precision):
    p = make_params(37, 23, precision=precision)
    rng = np.random.default_rng(1)
    rho = 1.1 + 0.3 * rng.random((23, 37))
    ux, uy = 0.05 * rng.standard_normal((2, 23, 37))
    run = lbm.Run(p, rho, ux, uy)
    f = run.get_f()
    ref = o.init(oracle_params(p), rho, ux, uy)
    assert rel_err(f, ref) < (1e-15 if precision == 0 else 1e-7)
    r, vx, vy = run.moments()
    tol = 1e-14 if precision == 0 else 2e-7
    np.testing.assert_allclose(r, rho, rtol=tol)
    np.testing.assert_allclose(vx, ux, atol=tol)
    np.testing.assert_allclose(vy, uy, atol=tol)


@pytest.mark.parametrize("precision", [0, 1])
def test_set_get_roundtrip(precision):
    p = make_params(70, 11, precision=precision)
    f = random_state(p, 2)
    run = lbm.Run(p, 1.0, 0.0, 0.0)
    run.set_f(f)
    g = run.get_f()
    if precision == 0:
        assert np.array_equal(f, g)
    else:
        assert rel_err(g, f) < 1e-7


# ------------------------------------------------------------ one-step parity

SIZES = [(16, 16), (64, 64), (96, 64), (61, 37), (130, 9)]


@pytest.mark.parametrize("Lx,Ly", SIZES)
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("reg", [0, 1])
@pytest.mark.parametrize("bc", [0, 1])
def test_one_step_fp64(Lx, Ly, scheme, reg, bc):
    p = make_params(Lx, Ly, scheme, reg, bc)
    f = random_state(p, 10 + Lx + 3 * Ly + scheme)
    got = gpu_step_from(p, f)
    ref = o.step(oracle_params(p), f)
    assert rel_err(got, ref) < F64_STEP


@pytest.mark.parametrize("Lx,Ly", [(64, 64), (61, 37)])
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("reg", [0, 1])
@pytest.mark.parametrize("bc", [0, 1])
def test_one_step_fp32dev(Lx, Ly, scheme, reg, bc):
    p = make_params(Lx, Ly, scheme, reg, bc, precision=1)
    f = random_state(p, 20 + Lx + scheme)
    got = gpu_step_from(p, f)
    # the oracle steps the same FP32-rounded state the GPU holds
    run = lbm.Run(p, 1.0, 0.0, 0.0)
    run.set_f(f)
    f_stored = run.get_f()
    ref = o.step(oracle_params(p), f_stored)
    assert rel_err(got, ref) < F32_STEP


def test_stochastic_rounding_statistics():
    """One FP32 step of a 64 x 64 state (CTU2, 65k stored values), once with
    round to nearest (r) and with 32 rounding seeds (the run reopened at 32
    step counts).  Stochastic rounding returns one of the two floats around
    the kernel's FP64 value x, so every outcome is r or the neighbour of r on
    the side of x (never both neighbours); it takes that neighbour with
    probability |x - r| / spacing <= 1/2, 1/4 on average over values, and is
    unbiased, so outcomes average to x.  The seed changes with the step."""
    import torch
    p = make_params(64, 64, precision=1, rounding=lbm.ROUND_NEAREST)
    f = random_state(p, 31)
    r = gpu_step_from(p, f)
    q = make_params(64, 64, precision=1, rounding=lbm.ROUND_STOCHASTIC)
    run = lbm.Run(q, 1.0, 0.0, 0.0)
    run.set_f(f)
    ws = run.ws.clone()
    torch.cuda.synchronize()
    run.close()
    outs = []
    for m in range(32):
        # state in field 0, seed from step 2m; a copy each time, because
        # reading the state back stages FP64 data through the other field
        rm = lbm.Run.attach(q, ws.clone(), 2 * m)
        rm.step(1)
        outs.append(rm.get_f())
        rm.close()
    w = o.velocity_set()[2][:, None, None] * q.rho_ref
    dr = (r - w).astype(np.float32)
    keep = np.abs(dr) > 1e-6                    # FP64 recovery of the stored FP32 value is exact here
    assert np.all(np.abs((r - w) - dr)[keep] < 0.01 * np.spacing(np.abs(dr[keep])))
    up, dn = np.nextafter(dr, np.float32(np.inf)), np.nextafter(dr, np.float32(-np.inf))
    k = []
    for g in outs:
        ds = (g - w).astype(np.float32)
        kk = np.where(ds == dr, 0, np.where(ds == up, 1, np.where(ds == dn, -1, 99)))
        assert not np.any(kk[keep] == 99), "stochastic result more than one float from nearest"
        k.append(kk[keep])
    k = np.array(k)
    assert not np.any((k == 1).any(axis=0) & (k == -1).any(axis=0)), "both neighbours taken"
    phat = (k != 0).mean(axis=0)
    assert k.shape[1] > 60000
    assert 0.22 < phat.mean() < 0.28
    assert (phat > 0.85).sum() <= 10
    assert abs(k.mean()) < 0.01
    assert (k[0] != k[1]).mean() > 0.1


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2])
def test_far_field_clamp_one_step(precision, scheme):
    """Density clamp outside the circle of radius R_BC (Sec. III B)."""
    p = make_params(90, 70, scheme, 0, 0, precision=precision, clamp_radius=24.5, clamp_rho=1.31)
    f = random_state(p, 90 + scheme)
    run = lbm.Run(p, 1.0, 0.0, 0.0)
    run.set_f(f)
    f_stored = run.get_f()
    run.step(1)
    got = run.get_f()
    run.close()
    ref = o.step(oracle_params(p), f_stored)
    assert rel_err(got, ref) < (F64_STEP if precision == 0 else F32_STEP)
    y, x = np.mgrid[0:70, 0:90]
    out = (x - 44.5) ** 2 + (y - 34.5) ** 2 > 24.5 ** 2
    np.testing.assert_allclose(got.sum(axis=0)[out], 1.31, rtol=1e-13 if precision == 0 else 1e-6)


def test_bubble_with_clamp_fp64_many_steps():
    """A vapour bubble in a clamped superheated liquid, 400 steps, FP64."""
    w = I.quiescent_bubble(80, radius=10.0)
    rho, ux, uy = w.fields()
    p = lbm.Params.from_workload(w, clamp_radius=30.0, clamp_rho=w.rho_ext)
    run = lbm.Run(p, rho, ux, uy)
    run.step(400)
    got = run.get_f()
    op = oracle_params(p)
    ref = o.run(op, o.init(op, rho, ux, uy), 400)
    assert rel_err(got, ref) < 1e-10


@pytest.mark.parametrize("Lx,Ly", [(1, 1), (1, 6), (2, 3), (5, 1), (55, 4), (56, 2), (57, 3), (63, 5), (64, 3),
                                   (65, 7), (111, 2), (112, 5), (113, 1), (200, 1)])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_one_step_edge_sizes(Lx, Ly, bc, precision):
    """Lattices narrower than a wavefront, ragged last strips, a single row or
    column; FP32 in its default launch (a pair of wavefronts per strip)."""
    p = make_params(Lx, Ly, 2, 0, bc, precision=precision)
    f = random_state(p, 30 + Lx + Ly)
    got = gpu_step_from(p, f)
    if precision:
        run = lbm.Run(p, 1.0, 0.0, 0.0)
        run.set_f(f)
        f = run.get_f()   # the FP32-stored state the GPU stepped
        run.close()
    ref = o.step(oracle_params(p), f)
    assert rel_err(got, ref) < (F64_STEP if precision == 0 else F32_STEP)


@pytest.mark.parametrize("precision,launch", [(0, (1, 1)), (0, (3, 2)), (0, (7, 2)), (0, (64, 1)), (0, (256, 2)),
                                              (1, (1, 1)), (1, (7, 2)), (1, (33, 2)), (1, (168, 1)),
                                              (1, (1, 0)), (1, (7, 0)), (1, (32, 0)), (1, (200, 0))])
def test_launch_shape_does_not_change_results(precision, launch):
    """Chunking rows differently changes nothing beyond rounding (a row's
    position in the unrolled row loop may round a multiply-add differently);
    a fixed launch shape is bitwise reproducible."""
    p = make_params(130, 45, 2, 1, 1, precision=precision)
    f = random_state(p, 40)
    base = gpu_step_from(p, f, nsteps=3, launch=(16, 2))
    got = gpu_step_from(p, f, nsteps=3, launch=launch)
    assert rel_err(got, base) < (1e-14 if precision == 0 else 1e-6)
    assert np.array_equal(got, gpu_step_from(p, f, nsteps=3, launch=launch))


@pytest.mark.parametrize("precision,launch", [(0, (8, 2)), (1, (8, 0)), (1, (8, 1))])
@pytest.mark.parametrize("reg", [0, 1])
@pytest.mark.parametrize("bc", [0, 1])
def test_short_chunks_against_oracle(precision, launch, reg, bc):
    """CTU2 with eight rows per chunk (six chunks, the last one ragged):
    every chunk starts its row march afresh, so the values carried from row
    to row (upwind differences, limited slopes, stencil sums) are formed
    again at each chunk start; the step still equals the oracle's."""
    p = make_params(130, 45, 2, reg, bc, precision=precision)
    f = random_state(p, 50 + 2 * reg + bc)
    if precision:
        run = lbm.Run(p, 1.0, 0.0, 0.0)
        run.set_f(f)
        f = run.get_f()
        run.close()
    got = gpu_step_from(p, f, launch=launch)
    ref = o.step(oracle_params(p), f)
    assert rel_err(got, ref) < (F64_STEP if precision == 0 else F32_STEP)


@pytest.mark.parametrize("precision", [0, 1])
def test_rejects_four_waves_per_group(precision):
    """The step kernels hold 32 KiB of LDS per wavefront: four per workgroup
    are refused with LBM_EINVAL and the previous shape is kept; the pair
    launch (one advecting and one colliding wavefront per strip) is for FP32
    storage only."""
    run = lbm.Run(make_params(40, 20, precision=precision), 1.0, 0.0, 0.0)
    run.set_launch(16, 2)
    with pytest.raises(lbm.LbmError) as ei:
        run.set_launch(16, 4)
    assert ei.value.status == lbm.LBM_EINVAL
    assert tuple(run.get_launch()) == (16, 2)
    if precision == 0:
        with pytest.raises(lbm.LbmError):
            run.set_launch(16, lbm.PAIR)
        assert tuple(run.get_launch()) == (16, 2)
    else:
        run.set_launch(16, lbm.PAIR)
        assert tuple(run.get_launch()) == (16, lbm.PAIR)
    run.close()


# ------------------------------------------------------------ many steps

def test_flat_interface_small_config_fp64_parity():
    """64 x 64 flat interface (a = 9/49, b = 2/21, T = 0.9 T_c, tau = 0.8,
    CTU2, dt = ds/4), 1000 steps: FP64 GPU against the oracle."""
    w = I.flat_interface_small()
    p = lbm.Params.from_workload(w)
    rho, ux, uy = w.fields()
    run = lbm.Run(p, rho, ux, uy)
    run.step(w.steps)
    r, vx, vy = run.moments()
    op = oracle_params(p)
    f = o.run(op, o.init(op, rho, ux, uy), w.steps)
    rr, rx, ry = o.field_moments(op, f)
    e = field_errors(r, vx, vy, rr, rx, ry)
    print("flat interface 64^2, 1000 steps, FP64 GPU vs oracle:", e)
    assert e["rho_max"] < 1e-10 and e["u_max"] < 1e-9


def test_bubble_fp32dev_against_oracle():
    """Quiescent bubble (T = 0.95, rho_ext = 0.95 rho_L, R = 12) on 96 x 96 for
    600 steps: FP32 deviation storage against the FP64 oracle."""
    w = I.quiescent_bubble(96, radius=12.0)
    rho, ux, uy = w.fields()
    p = lbm.Params.from_workload(w, precision=lbm.FP32_DEV)
    run = lbm.Run(p, rho, ux, uy)
    run.step(600)
    r, vx, vy = run.moments()
    op = oracle_params(p)
    f = o.run(op, o.init(op, rho, ux, uy), 600)
    rr, rx, ry = o.field_moments(op, f)
    e = field_errors(r, vx, vy, rr, rx, ry)
    print("bubble 96^2, 600 steps, FP32-dev GPU vs oracle:", e)
    assert e["rho_max"] < 1e-5 and e["u_max"] < 1e-4


def test_sheared_bubble_regularized_fp64():
    p = lbm.Params(Lx=80, Ly=72, T=0.95, kappa=1.0, tau=0.7, regularize=1, bc_y=1, u_wall=0.02,
                   rho_wall=1.3886)
    rho = I.bubble(80, 72, 0.579, 1.3886, 10.0)
    ux, uy = I.shear_profile(80, 72, 2 * 0.02 / 72)
    run = lbm.Run(p, rho, ux, uy)
    run.step(300)
    got = run.get_f()
    op = oracle_params(p)
    ref = o.run(op, o.init(op, rho, ux, uy), 300)
    assert rel_err(got, ref) < 1e-10


# ------------------------------------------------------------ diagnostics

def test_reduce_matches_oracle_fp64():
    w = I.quiescent_bubble(150, radius=25.0)
    rho, ux, uy = w.fields()
    p = lbm.Params.from_workload(w)
    p.Lx, p.Ly = 150, 150
    run = lbm.Run(p, rho, ux, uy)
    run.step(5)
    f = run.get_f()
    thr = 0.5 * (w.rho_vapour + w.rho_liquid)
    st = run.reduce(thr)
    ref = o.reduce(oracle_params(p), f, thr)
    assert st["n_bubble"] == int(ref["n_bubble"]) and st["n_nonfinite"] == 0
    for k in ("mass", "sx", "sy", "sxx", "sxy", "syy"):
        assert st[k] == pytest.approx(ref[k], rel=1e-12, abs=1e-9), k
    for k in ("mom_x", "mom_y"):
        assert st[k] == pytest.approx(ref[k], abs=1e-10 * ref["mass"]), k
    assert st["A_rel"] == pytest.approx(ref["n_bubble"] / 150 ** 2)
    assert st["R_eq"] == pytest.approx(np.sqrt(ref["n_bubble"] / np.pi))


def test_reduce_ellipse_shape():
    """Gyration tensor of a synthetic elliptical bubble (semi-axes 40, 20,
    tilted 0.3 rad): a, b, D and theta to within lattice discretisation."""
    L = 200
    A, B, th = 40.0, 20.0, 0.3
    y, x = np.mgrid[0:L, 0:L].astype(float)
    x -= (L - 1) / 2
    y -= (L - 1) / 2
    xr = x * np.cos(th) + y * np.sin(th)
    yr = -x * np.sin(th) + y * np.cos(th)
    inside = (xr / A) ** 2 + (yr / B) ** 2 < 1
    rho = np.where(inside, 0.6, 1.4)
    p = lbm.Params(Lx=L, Ly=L)
    run = lbm.Run(p, rho, 0.0, 0.0)
    st = run.reduce(1.0)
    assert st["a"] == pytest.approx(A, rel=0.01)
    assert st["b"] == pytest.approx(B, rel=0.02)
    assert st["D"] == pytest.approx((A - B) / (A + B), abs=0.01)
    assert st["theta"] == pytest.approx(th, abs=0.01)
    assert st["cx"] == pytest.approx((L - 1) / 2, abs=0.05)


def test_reduce_reports_nonfinite():
    p = make_params(40, 30)
    f = random_state(p, 50)
    f[3, 7, 11] = np.nan
    f[9, 0, 0] = np.inf
    run = lbm.Run(p, 1.0, 0.0, 0.0)
    run.set_f(f)
    with pytest.raises(lbm.LbmError) as ei:
        run.reduce(1.0)
    assert ei.value.status == lbm.LBM_ENONFINITE
    st = run.reduce(1.0, allow_nonfinite=True)
    assert st["n_nonfinite"] == 2


# ------------------------------------------------------------ determinism, resume, batch

def test_bitwise_determinism():
    p = make_params(128, 96, 2, 0, 1, precision=1)
    f = random_state(p, 60)
    a = gpu_step_from(p, f, nsteps=20)
    b = gpu_step_from(p, f, nsteps=20)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", [0, 1])
def test_checkpoint_resume_bitwise(precision):
    """A copied workspace reopened at its step continues bitwise (FP32: the
    stochastic rounding seed follows the step count)."""
    import torch
    p = make_params(100, 64, 2, 0, 0, precision=precision)
    f = random_state(p, 70)
    run = lbm.Run(p, 1.0, 0.0, 0.0)
    run.set_f(f)
    run.step(9)
    ws_copy = run.ws.clone()
    torch.cuda.synchronize()
    run.step(11)
    end = run.get_f()
    resumed = lbm.Run.attach(p, ws_copy, 9)
    assert resumed.step_count == 9
    resumed.step(11)
    assert np.array_equal(resumed.get_f(), end)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("graph_steps", [0, 4])
def test_batch_equals_single_runs(graph_steps, precision):
    """Batched steps, plain or replayed from a captured graph, equal single
    runs bitwise (FP32: every replay advances the rounding seed as single steps do)."""
    specs = [make_params(70, 50, bc=1, precision=precision), make_params(33, 19, precision=precision),
             make_params(128, 64, bc=1, T=0.9, precision=precision)]
    states = [random_state(p, 80 + i) for i, p in enumerate(specs)]
    singles = [gpu_step_from(p, f, nsteps=9) for p, f in zip(specs, states)]
    batch = lbm.Batch(specs, [(1.0, 0.0, 0.0)] * len(specs))
    for m, f in zip(batch.runs, states):
        m.set_f(f)
    batch.step(5, graph_steps=graph_steps)
    batch.step(4, graph_steps=graph_steps)
    for m, ref in zip(batch.runs, singles):
        assert m.step_count == 9
        assert np.array_equal(m.get_f(), ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_set_launch_and_autotune(precision):
    """A batch re-chunked to another rows-per-wavefront still equals single
    runs with that launch shape; the autotuner keeps one of its candidates
    (and, for FP32, one of the two launch modes) and its trial steps advance
    every member."""
    specs = [make_params(70, 50, bc=1, precision=precision), make_params(33, 19, precision=precision)]
    states = [random_state(p, 95 + i) for i, p in enumerate(specs)]
    singles = [gpu_step_from(p, f, nsteps=3, launch=(5, 1)) for p, f in zip(specs, states)]
    batch = lbm.Batch(specs, [(1.0, 0.0, 0.0)] * len(specs))
    for m, f in zip(batch.runs, states):
        m.set_f(f)
    batch.set_launch(5)
    batch.step(3, graph_steps=2)
    for m, ref in zip(batch.runs, singles):
        assert np.array_equal(m.get_f(), ref)
    rows = batch.autotune(1)
    assert rows in (16, 24, 32, 40, 48, 64, 96, 128, 192, 256)
    # 10 common candidates per launch mode (one mode for FP64, two for
    # FP32, persistent trials of 1 + 16 steps), one re-timing, up to 4 per
    # class (two classes) in the chosen mode
    common = 10 * 2 + (0 if precision == 0 else 10 * 17)
    per = 17 if batch.mode == lbm.BATCH_PERSISTENT else 2
    counts = {m.step_count for m in batch.runs}
    assert len(counts) == 1 and 3 + common + per <= counts.pop() <= 3 + common + 9 * per
    assert batch.mode in ((lbm.BATCH_PER_STEP,) if precision == 0 else (lbm.BATCH_PER_STEP, lbm.BATCH_PERSISTENT))
    per_run = [m.get_launch()[0] for m in batch.runs]
    assert all(r in (rows, rows // 2, (3 * rows) // 4, (3 * rows) // 2, 2 * rows) for r in per_run)
    st = batch.runs[0].reduce(1.0)
    assert st["n_nonfinite"] == 0
    # the per-class choice stays bit-exact against single runs with that shape
    states = [random_state(p, 97 + i) for i, p in enumerate(specs)]
    at = batch.runs[0].step_count
    singles = [gpu_step_from(p, f, nsteps=3, launch=(r, 1), start_step=at) for p, f, r in zip(specs, states, per_run)]
    for m, f in zip(batch.runs, states):
        m.set_f(f)
    batch.step(3, graph_steps=3)
    batch.sync_status()
    for m, ref in zip(batch.runs, singles):
        assert np.array_equal(m.get_f(), ref)
    batch.close()
    # a later batch of the same shapes starts from the tuned values
    again = lbm.Batch(specs, [(1.0, 0.0, 0.0)] * len(specs))
    assert [m.get_launch()[0] for m in again.runs] == per_run
    again.close()


PERSIST_SPECS = {
    # (Lx, Ly, walls): ragged strips and chunks, a single-item lattice, and
    # lattices whose last chunk is shorter than the 4-row reach of a step
    "mixed": [(70, 50, 1), (33, 19, 0), (128, 64, 1), (9, 7, 0), (57, 130, 0), (200, 66, 1)],
    "periodic": [(33, 19, 0), (9, 7, 0), (57, 130, 0), (120, 121, 0)],
    "walls": [(70, 50, 1), (128, 64, 1), (40, 9, 1)],
}


@pytest.mark.parametrize("rows", [5, 64])
@pytest.mark.parametrize("graph_steps", [0, 6])
@pytest.mark.parametrize("kinds", sorted(PERSIST_SPECS))
def test_persistent_batch_equals_single_runs(kinds, graph_steps, rows):
    """The persistent batched launch (FP32: one launch for up to 64 steps,
    each work item waiting only for its neighbours of the previous step)
    equals single runs bitwise over 150 steps: periodic and wall runs in one
    launch, rows per item down to 5 (chunks of 2 rows at the lattice edge),
    several launches (the 64-step bound crossed at odd parity), and launches
    replayed from a captured graph."""
    specs = [make_params(Lx, Ly, bc=bc, precision=1) for Lx, Ly, bc in PERSIST_SPECS[kinds]]
    states = [random_state(p, 300 + i) for i, p in enumerate(specs)]
    singles = [gpu_step_from(p, f, nsteps=150) for p, f in zip(specs, states)]
    batch = lbm.Batch(specs, [(1.0, 0.0, 0.0)] * len(specs))
    batch.set_launch(rows)
    batch.set_mode(lbm.BATCH_PERSISTENT)
    assert batch.mode == lbm.BATCH_PERSISTENT
    for m, f in zip(batch.runs, states):
        m.set_f(f)
    batch.step(71, graph_steps=graph_steps)
    batch.step(79, graph_steps=graph_steps)
    batch.sync_status()
    for m, ref in zip(batch.runs, singles):
        assert m.step_count == 150
        got = m.get_f()
        assert np.all(np.isfinite(ref))
        assert np.array_equal(got, ref)
    # switching back continues the same trajectory
    more = [gpu_step_from(p, ref, nsteps=3, start_step=150) for p, ref in zip(specs, singles)]
    for m, ref in zip(batch.runs, singles):
        m.set_f(ref)
    batch.set_mode(lbm.BATCH_PER_STEP)
    batch.step(3)
    for m, ref in zip(batch.runs, more):
        assert np.array_equal(m.get_f(), ref)
    batch.close()


@pytest.mark.parametrize("scheme,reg", [(1, 0), (1, 1), (2, 1)])
def test_persistent_batch_other_schemes(scheme, reg):
    """The persistent launch's other instantiations (CTU1, regularized)
    equal single runs bitwise over 70 steps, periodic and wall runs mixed."""
    specs = [make_params(Lx, Ly, scheme=scheme, reg=reg, bc=bc, precision=1)
             for Lx, Ly, bc in ((70, 50, 1), (33, 19, 0), (57, 66, 0))]
    states = [random_state(p, 500 + i) for i, p in enumerate(specs)]
    singles = [gpu_step_from(p, f, nsteps=70) for p, f in zip(specs, states)]
    batch = lbm.Batch(specs, [(1.0, 0.0, 0.0)] * len(specs))
    batch.set_launch(8)
    batch.set_mode(lbm.BATCH_PERSISTENT)
    for m, f in zip(batch.runs, states):
        m.set_f(f)
    batch.step(70, graph_steps=10)
    batch.sync_status()
    for m, ref in zip(batch.runs, singles):
        assert np.array_equal(m.get_f(), ref)
    batch.close()


def test_persistent_batch_reports_a_wait_past_its_bound():
    """A dependency wait that exceeds its bound ends the launch with an
    error instead of hanging: with a bound of one poll, the item of step 1
    of a one-item batch gives up while step 0 still runs, and the status
    call reports it; the default bound then gives exact results again."""
    p = make_params(40, 40, precision=1)
    f = random_state(p, 321)
    batch = lbm.Batch([p], [(1.0, 0.0, 0.0)])
    batch.set_launch(64)
    batch.set_mode(lbm.BATCH_PERSISTENT)
    batch.set_wait_limit(1)
    batch.runs[0].set_f(f)
    batch.step(8)
    with pytest.raises(lbm.LbmError) as ei:
        batch.sync_status()
    assert ei.value.status == lbm.LBM_EDEVICE
    batch.sync_status()  # the error word was cleared
    batch.set_wait_limit(0)
    batch.runs[0].set_f(f)
    batch.step(8)
    batch.sync_status()
    assert np.array_equal(batch.runs[0].get_f(), gpu_step_from(p, f, nsteps=8, start_step=8))
    batch.close()


def test_boundary_batch_aliases():
    """lbm_step_batch (graph-replayed steps) equals lbm_batch_step, and
    lbm_init_batch builds the same batch as lbm_batch_init."""
    import ctypes
    specs = [make_params(70, 50, bc=1, precision=1), make_params(33, 19, precision=1)]
    states = [random_state(p, 400 + i) for i, p in enumerate(specs)]
    a = lbm.Batch(specs, [(1.0, 0.0, 0.0)] * len(specs))
    b = lbm.Batch(specs, [(1.0, 0.0, 0.0)] * len(specs))
    for x, y, f in zip(a.runs, b.runs, states):
        x.set_f(f)
        y.set_f(f)
    a.step(45)
    stream = ctypes.c_void_p(b.torch.cuda.current_stream().cuda_stream)
    assert lbm.LIB.lbm_step_batch(b.handle, 45, stream) == lbm.LBM_OK
    for x, y in zip(a.runs, b.runs):
        assert y.step_count == 45
        assert np.array_equal(x.get_f(), y.get_f())
    a.close()
    b.close()
    n = len(specs)
    cp = (lbm.CParams * n)(*[p.c() for p in specs])
    ws = b.torch.empty(int(lbm.LIB.lbm_batch_workspace_bytes(n, cp)), dtype=b.torch.uint8, device="cuda")
    arrs = [np.full((p.Ly, p.Lx), 1.1) for p in specs] + [np.zeros((p.Ly, p.Lx)) for p in specs]
    P = ctypes.POINTER(ctypes.c_double)
    rho = (P * n)(*[a_.ctypes.data_as(P) for a_ in arrs[:n]])
    zero = (P * n)(*[a_.ctypes.data_as(P) for a_ in arrs[n:]])
    h = ctypes.c_void_p()
    assert lbm.LIB.lbm_init_batch(n, cp, ctypes.c_void_p(ws.data_ptr()), ws.numel(), stream, rho, zero, zero,
                                  ctypes.byref(h)) == lbm.LBM_OK
    assert lbm.LIB.lbm_step_batch(h, 2, stream) == lbm.LBM_OK
    lbm.LIB.lbm_batch_destroy(h)


def test_persistent_mode_needs_fp32():
    batch = lbm.Batch([make_params(33, 19, precision=0)], [(1.0, 0.0, 0.0)])
    with pytest.raises(lbm.LbmError) as ei:
        batch.set_mode(lbm.BATCH_PERSISTENT)
    assert ei.value.status == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError):
        batch.set_mode(7)
    assert batch.mode == lbm.BATCH_PER_STEP
    batch.close()


def test_rejects_bad_parameters():
    p = make_params(16, 16)
    p.dt = 0.5
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Run(p, 1.0, 0.0, 0.0)
    assert ei.value.status == lbm.LBM_ECFL
    p = make_params(16, 16)
    with pytest.raises(lbm.LbmError):
        lbm.Run(p, np.full((16, 16), 4.0), 0.0, 0.0)  # beyond 1/b
    with pytest.raises(lbm.LbmError):
        lbm.Run(p, np.full((16, 16), np.nan), 0.0, 0.0)


def test_fp32dev_ten_thousand_steps_against_oracle():
    """FP32-deviation storage against the FP64 oracle after 10^4 steps
    (quiescent bubble, T = 0.95, rho_ext = 0.95 rho_L, R = 14, 96 x 96
    periodic, CTU2): rho and u (u error normalised by the largest |u|) within
    1e-5 with stochastic rounding, for the storage reference of the workloads
    (the far liquid's density) and for one midway between the phases.  Round
    to nearest is reported beside them: its errors repeat step after step
    where the flow is nearly steady and add up coherently, so it is bounded
    at 5e-5 and 1e-4 only."""
    w = I.quiescent_bubble(96, radius=14.0)
    rho, ux, uy = w.fields()
    op = None
    errs = {}
    cases = (("far liquid, stochastic", w.rho_ext, lbm.ROUND_STOCHASTIC),
             ("midway, stochastic", 0.5 * (w.rho_vapour + w.rho_ext), lbm.ROUND_STOCHASTIC),
             ("far liquid, nearest", w.rho_ext, lbm.ROUND_NEAREST))
    for name, rho_ref, rounding in cases:
        p = lbm.Params.from_workload(w, precision=lbm.FP32_DEV, rounding=rounding, rho_ref=rho_ref)
        run = lbm.Run(p, rho, ux, uy)
        run.step(10000)
        r, vx, vy = run.moments()
        run.close()
        if op is None:
            op = oracle_params(p)
            f = o.run(op, o.init(op, rho, ux, uy), 10000)
            rr, rx, ry = o.field_moments(op, f)
        errs[name] = field_errors(r, vx, vy, rr, rx, ry)
        print("bubble 96^2, 10^4 steps, FP32-dev GPU vs oracle, rho_ref %s:" % name, errs[name])
    for name in ("far liquid, stochastic", "midway, stochastic"):
        e = errs[name]
        assert e["rho_max"] < 1e-5 and e["u_max"] < 1e-5, name
    e = errs["far liquid, nearest"]
    assert e["rho_max"] < 5e-5 and e["u_max"] < 1e-4


# ------------------------------------------------- full-size sampled parity

def sampled_regions_step(p, rho, ux, uy, launch, boxes):
    """One step of a full-size run in the given launch shape; for each box
    (j0, j1, i0, i1) the GPU output is compared with the oracle's step of a
    cut of the GPU's own input state around the box (gpu_helpers.box_rows,
    oracle_box_step).  Returns the largest error relative to max |f| of each box."""
    import torch
    run = lbm.Run(p, rho, ux, uy)
    run.set_launch(*launch)
    Ly, Lx = p.Ly, p.Lx
    cuts = []
    fin = run.get_f_device()
    for box in boxes:
        r0, r1 = box_rows(box, Ly, p.bc_y)
        cols = torch.arange(box[2] - 4, box[3] + 4, device="cuda") % Lx
        rows = torch.arange(r0, r1, device="cuda") % Ly
        cuts.append((r0, fin.index_select(1, rows).index_select(2, cols).cpu().numpy()))
    del fin
    torch.cuda.synchronize()
    run.step(1)
    fout = run.get_f_device()
    errs = []
    op = oracle_params(p)
    for box, (r0, fcut) in zip(boxes, cuts):
        j0, j1, i0, i1 = box
        got = fout[:, j0:j1, :].index_select(2, torch.arange(i0, i1, device="cuda") % Lx).cpu().numpy()
        errs.append(rel_err(got, oracle_box_step(op, fcut, box, r0, Ly, p.bc_y)))
    run.close()
    return errs


def large_boxes(L, strip=56, rows=168):
    c = L // 2
    last_strip = ((L - 1) // strip) * strip   # start of the last (ragged) strip
    last_chunk = ((L - 1) // rows) * rows     # start of the last chunk
    return [
        (0, 10, 0, 10),                                  # corner: periodic wrap in x and y
        (L - 10, L, L - 10, L),                          # opposite corner, ragged last strip and chunk
        (c - 64, c - 52, c - 6, c + 6),                  # bubble interface (radius 60)
        (c - 6, c + 6, c + 55, c + 67),
        (rows - 6, rows + 6, strip - 6, strip + 6),      # chunk and strip boundaries
        (5 * rows - 5, 5 * rows + 7, 7 * strip - 7, 7 * strip + 5),
        (last_chunk - 6, last_chunk + 6, last_strip - 6, last_strip + 6),
    ]


@pytest.mark.parametrize("precision,launch", [(1, (32, 0)), (1, (40, 0)), (1, (168, 1)), (0, (168, 2))])
def test_full_size_6144_sampled_against_oracle(precision, launch):
    """The 6144 x 6144 benchmark workload (bubble of radius 60, T = 0.95) in
    the launch shapes the benchmark times (the autotuner picks the pair
    launch at 32 or 40 rows for FP32, 168 x 2 for FP64): one step, seven
    sampled boxes (wrapped corners, the bubble interface, strip boundaries
    and the chunk boundaries of that launch, the ragged last strip and
    chunk) against the oracle."""
    w = I.large_lattice(6144)
    rho, ux, uy = w.fields()
    p = lbm.Params.from_workload(w, precision=precision)
    errs = sampled_regions_step(p, rho, ux, uy, launch, large_boxes(6144, rows=launch[0]))
    print("6144^2 precision %d launch %s: box errors" % (precision, launch), ["%.1e" % e for e in errs])
    assert max(errs) < (F64_STEP if precision == 0 else F32_STEP)


def test_full_size_2048_sheared_sampled_against_oracle():
    """The 2048 x 2048 sheared workload (walls moving at -+u_w, shear rate
    1e-4, noise, FP32) in its default launch shape: boxes at both walls and
    in the interior against the oracle."""
    w = I.sheared_bubble(1e-4, 2048)
    rho, ux, uy = w.fields()
    p = lbm.Params.from_workload(w, precision=lbm.FP32_DEV)
    boxes = [(0, 8, 0, 10), (2040, 2048, 2038, 2048), (0, 8, 1000, 1012), (2040, 2048, 55, 67),
             (1000, 1012, 1020, 1032), (990, 1002, 1020 + 30, 1032 + 30)]
    run = lbm.Run(p, rho, ux, uy)
    launch = tuple(run.get_launch())
    run.close()
    errs = sampled_regions_step(p, rho, ux, uy, launch, boxes)
    print("2048^2 sheared launch %s: box errors" % (launch,), ["%.1e" % e for e in errs])
    assert max(errs) < F32_STEP


@pytest.mark.parametrize("precision", [1, 0])
def test_maximum_size_8192_sampled_against_oracle(precision):
    """The largest lattices a run accepts, 8192 x 8192 = 2^26 nodes with FP32
    storage and 8192 x 8191 with FP64 storage (eight FP64 planes must span
    fewer than 2^32 bytes, the range of one buffer descriptor), with the
    bubble workload's fluid: one step in the default launch shape, sampled
    boxes (wrapped corners, the ragged last strip of 16 columns, the bubble
    interface) against the oracle.  At 8192 x 8192 in FP64 the last value of
    planes 7 and 15 would lie outside the descriptor's range."""
    w = I.quiescent_bubble(8192, radius=60.0)
    if precision == 0:
        w = w.with_size(8192, 8191)
    rho, ux, uy = w.fields()
    p = lbm.Params.from_workload(w, precision=precision)
    run = lbm.Run(p, 1.0, 0.0, 0.0)
    launch = tuple(run.get_launch())
    run.close()
    c = 4096
    Ly = w.Ly
    boxes = [(0, 8, 0, 8), (Ly - 8, Ly, 8180, 8192), (c - 66, c - 56, c - 5, c + 5), (2000, 2010, 8170, 8186)]
    errs = sampled_regions_step(p, rho, ux, uy, launch, boxes)
    print("8192^2 precision %d launch %s: box errors" % (precision, launch), ["%.1e" % e for e in errs])
    assert max(errs) < (F64_STEP if precision == 0 else F32_STEP)


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("dt_case", ["cfl", "small"])
def test_degenerate_time_steps(scheme, bc, dt_case):
    """Degenerate Courant numbers, FP64, 20 steps against the oracle: dt at
    the CFL limit of Sec. II C 1 (nu |xi| = 1 for the fast components, whose
    upwind update is then an exact shift and whose limited corrections
    vanish), and a small dt = 1/64 with tau = dt/2 + 0.01, close to the
    vanishing viscosity T (tau - dt/2) of the split scheme."""
    ql = (3 + 6 ** 0.5) ** 0.5
    if dt_case == "cfl":
        p = make_params(70, 45, scheme, 0, bc, dt=1.0 / ql)
    else:
        p = make_params(70, 45, scheme, 0, bc, dt=1.0 / 64, tau=1.0 / 128 + 0.01)
    f = random_state(p, 150 + scheme + 2 * bc)
    got = gpu_step_from(p, f, nsteps=20)
    ref = o.run(oracle_params(p), f.copy(), 20)
    assert rel_err(got, ref) < 1e-12


def test_fp32dev_sheared_ten_thousand_steps_against_fp64():
    """FP32-deviation storage with moving walls (sheared bubble, 192 x 192,
    shear rate 1e-4, radius 20, T = 0.95) against the FP64 stepper, which
    follows the oracle to 1e-10 over long runs with walls: rho and u (u error
    normalised by the largest |u|) within 1e-5 after 10^4 steps (measured
    2.8e-6 and 3.5e-6)."""
    w = I.sheared_bubble(1e-4, 192).with_size(192, 192, radius=20.0)
    rho, ux, uy = w.fields()
    r64 = lbm.Run(lbm.Params.from_workload(w, precision=lbm.FP64), rho, ux, uy)
    r32 = lbm.Run(lbm.Params.from_workload(w, precision=lbm.FP32_DEV), rho, ux, uy)
    r64.step(10000)
    r32.step(10000)
    a, b = r64.moments(), r32.moments()
    r64.close()
    r32.close()
    e = field_errors(b[0], b[1], b[2], a[0], a[1], a[2])
    print("sheared 192^2, 10^4 steps, FP32-dev vs FP64:", e)
    assert e["rho_max"] < 1e-5 and e["u_max"] < 1e-5
