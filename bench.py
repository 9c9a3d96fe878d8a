"""Throughput of the CTU lattice Boltzmann step on one MI355X.

Workload (default): the paper's largest lattice, 6144 x 6144 periodic, a van
der Waals fluid at T = 0.95 T_c (a = 9/8, b = 1/3), superheated liquid at
0.95 rho_L with a vapour bubble of radius 60 nodes, tau = 0.7, kappa = 1,
CTU2, ds = 1, dt = 1/4.  One step = one pass of the fused kernel over the
whole lattice (moments, equilibrium, van der Waals force with its 25-point
stencils, BGK, CTU2 advection).  The headline value is the FP32-deviation
stepper's MLUPS; the FP64 stepper runs on the same input for the speedup
and for the rho/u error of the FP32 storage.

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
VALU_SIMDS, CLOCK_HZ = 256 * 4, 2.4e9   # MI355X: 256 CUs x 4 SIMDs, peak engine clock
BYTES_PER_LUP = {"f32": 128.0, "f64": 256.0}  # read + write 16 distributions once


def kernel_source_hash():
    h = hashlib.sha256()
    for n in ("lbm_kernels.hip", "lbm_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1802_01272_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profiled(kernel_key, launch):
    """The committed rocprofv3 counter summary (profiles/traffic.json) of a
    step kernel in one launch shape, if it was taken on the current kernel
    source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = t.get(kernel_key)
    if not entry or entry.get("source_hash") != kernel_source_hash():
        return None
    return entry.get("by_launch", {}).get("%d,%d" % tuple(launch))


def measured_valu(kernel_key, launch):
    """VALU instructions per launch (rocprofv3 SQ_INSTS_VALU), or None."""
    e = _profiled(kernel_key, launch)
    return e.get("valu_per_launch") if e else None


def measured_traffic(kernel_key, launch):
    """HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a
    plain copy's reading), or None."""
    e = _profiled(kernel_key, launch)
    return e.get("bytes_per_launch") if e else None


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(workload, rho, ux, uy, budget_s=12.0, rows=256, max_steps=20, single_budget_s=6.0):
    """The oracle (FP64 CPU reference, OpenMP) timed on a band of `rows` full
    rows of the workload's initial state (periodic), one step at a time until
    about budget_s seconds of work on all its threads, then again on one
    thread for about single_budget_s seconds."""
    import numpy as np
    import oracle as o
    p = o.Params(Lx=workload.Lx, Ly=rows, ds=workload.ds, dt=workload.dt, tau=workload.tau, T=workload.T,
                 a=workload.a, b=workload.b, kappa=workload.kappa, scheme=workload.scheme,
                 regularize=workload.regularize)
    j0 = (workload.Ly - rows) // 2
    f = o.init(p, np.ascontiguousarray(rho[j0:j0 + rows]), np.ascontiguousarray(ux[j0:j0 + rows]),
               np.ascontiguousarray(uy[j0:j0 + rows]))
    o.step(p, f)  # first touch / warm-up
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps:
        f = o.step(p, f)
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    threads = o.num_threads()
    # the same band on one thread
    o.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        steps1 = 0
        while steps1 < max_steps:
            f = o.step(p, f)
            steps1 += 1
            if time.perf_counter() - t1 > single_budget_s:
                break
        dt1 = time.perf_counter() - t1
    finally:
        o.set_num_threads(threads)
    return {"value": round(p.Lx * p.Ly * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "cpu": cpu_model(),
            "single_thread": {"value": round(p.Lx * p.Ly * steps1 / dt1 / 1e6, 3), "unit": "MLUPS", "steps": steps1},
            "sample": "%d x %d band of the workload's initial state (periodic), %d steps, FP64" % (p.Lx, rows, steps)}


def timed_steps(torch, fn, steps):
    """Device milliseconds of fn(steps), HIP events on torch's current stream
    (the stream the library launches on)."""
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def batched_sweep(args, torch, I, lbm, graph_steps=20):
    """Aggregate MLUPS of the 32-run sweep (lattice edges 256..1536, T/T_c in
    [0.85, 0.97], shear rates 0, 1e-5, 1e-4, FP32 deviation storage): one
    batched launch per step, replayed from a HIP graph, rows per wavefront
    from the batch autotuner; against the same runs stepped one after another,
    each with its own autotuned launch shape."""
    sweep = I.batched_sweep(32, seed=5)
    params = [lbm.Params.from_workload(w, precision=lbm.FP32_DEV) for w in sweep]
    fields = [w.fields() for w in sweep]
    nodes = sum(w.Lx * w.Ly for w in sweep)
    steps = args.steps
    batch = lbm.Batch(params, fields)
    rows = batch.autotune(2)
    mode = "persistent" if batch.mode == lbm.BATCH_PERSISTENT else "per_step"
    # the warm-up captures and replays the graph, so no capture is timed
    batch.step(max(args.warmup, 2 * graph_steps + 1), graph_steps=graph_steps)
    ms_batch = timed_steps(torch, lambda n: batch.step(n, graph_steps=graph_steps), steps)
    batch.sync_status()
    batch.close()
    del batch
    torch.cuda.empty_cache()
    ms_seq = 0.0
    for p, (rho, ux, uy) in zip(params, fields):
        launch = lbm.autotune(p, steps_per_trial=2)
        run = lbm.Run(p, rho, ux, uy)
        run.set_launch(*launch)
        run.step(args.warmup)
        ms_seq += timed_steps(torch, run.step, steps)
        run.close()
    value = nodes * steps / (ms_batch * 1e-3) / 1e6
    seq = nodes * steps / (ms_seq * 1e-3) / 1e6
    return {"metric": "aggregate MLUPS, batched sweep vs the same runs sequentially", "value": round(value, 1),
            "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
            "ms_per_step": round(ms_batch / steps, 5), "higher_is_better": True, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "batched_sweep_32", "runs": len(sweep), "nodes": nodes,
                       "edges": sorted({w.Lx for w in sweep}), "rows_per_wave": rows, "graph_steps": graph_steps,
                       "mode": mode,
                       "storage": "FP32 f - w rho_ref"},
            "sequential": {"value": round(seq, 1), "ms_per_step": round(ms_seq / steps, 5)},
            "speedup_batched_over_sequential": round(ms_seq / ms_batch, 3)}


def batched_tail(args, torch, I, lbm, graph_steps=20, copies=(1, 2, 4)):
    """What the launch boundary costs the batched sweep: the 32-run sweep, and
    the same sweep held 2 and 4 times over in one batch (every run repeated),
    each autotuned on itself, then timed in both launch modes with the tuned
    rows: one launch per step, and the persistent launch (no boundary
    between steps).  A straight-line fit of the time per step against the
    number of copies n, T(n) = c + n m, splits a step into the part that
    grows with the work (m per copy) and the part that does not (c): the
    launch itself and the tail in which the step's last items run on a
    partly idle chip."""
    import numpy as np
    sweep = I.batched_sweep(32, seed=5)
    params = [lbm.Params.from_workload(w, precision=lbm.FP32_DEV) for w in sweep]
    fields = [w.fields() for w in sweep]
    nodes = sum(w.Lx * w.Ly for w in sweep)
    modes = {"per_step": lbm.BATCH_PER_STEP, "persistent": lbm.BATCH_PERSISTENT}
    ms = {name: {} for name in modes}
    tuned = {}
    for n in copies:
        batch = lbm.Batch(params * n, fields * n)
        batch.autotune(2)
        tuned[n] = {"mode": [k for k, v in modes.items() if v == batch.mode][0],
                    "rows": sorted({m.get_launch()[0] for m in batch.runs})}
        for name, mode in modes.items():
            batch.set_mode(mode)
            batch.step(max(args.warmup, 2 * graph_steps + 1), graph_steps=graph_steps)
            t = timed_steps(torch, lambda k: batch.step(k, graph_steps=graph_steps), args.steps) / args.steps
            batch.sync_status()
            ms[name][n] = t
            print("[bench] batched sweep x%d, %s: %.5f ms per step" % (n, name, t), file=sys.stderr, flush=True)
        batch.close()
        del batch
        torch.cuda.empty_cache()
    fits = {}
    for name in modes:
        ns = np.array(sorted(ms[name]), dtype=float)
        ts = np.array([ms[name][int(n)] for n in ns])
        m, c = np.polyfit(ns, ts, 1)
        fits[name] = {"fixed_ms": round(float(c), 5), "per_copy_ms": round(float(m), 5),
                      "marginal_mlups": round(nodes / (float(m) * 1e-3) / 1e6, 1),
                      "ms_per_step": {str(n): round(ms[name][n], 5) for n in sorted(ms[name])},
                      "mlups": {str(n): round(n * nodes / (ms[name][n] * 1e-3) / 1e6, 1) for n in sorted(ms[name])}}
    return {"metric": "batched sweep: per-step time against copies of the sweep held in one batch",
            "value": round(fits["per_step"]["fixed_ms"] / ms["per_step"][1], 4),
            "unit": "fixed part of one copy's step (one launch per step)",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": False,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "batched_sweep_32", "runs": len(sweep), "nodes": nodes,
                       "copies": list(copies), "graph_steps": graph_steps, "autotuned": tuned},
            "modes": fits}


def copy_probe(args, torch):
    """Memory-side ceilings of the step's access shape on the 16-plane FP32
    field of args.L^2 nodes: plain copies (no arithmetic) that move the step's
    algorithmic bytes (read and write every distribution once) in the step's
    strip-marching pattern and in simpler ones; GB/s of algorithmic bytes,
    HIP events, best and median of `reps` launches each."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1802_01272_amd", "_lib", "libprobe.so"))
    lib.probe_strip_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 6 + [ctypes.c_void_p]
    lib.probe_flat_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    lib.probe_blocked_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p] + [ctypes.c_int] * 5 + [ctypes.c_void_p]
    L, reps = args.L, 20
    n = 16 * L * L
    nblk = 16 * ((L + 55) // 56) * 56 * L  # the strip-blocked variants' field
    src = torch.empty(max(n, nblk), dtype=torch.float32, device="cuda").uniform_()
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    algo = 2.0 * 4 * n
    variants = []
    # (name, outw, rows, halo_y, lds bytes per workgroup); 36 KiB of LDS holds
    # a CU to 4 wavefronts, the number of loading wavefronts of the step's
    # pair launch
    for outw, hy, rows, lds in ((56, 4, 32, 0), (56, 4, 32, 36864), (56, 0, 32, 0), (64, 4, 32, 0),
                                (64, 4, 32, 36864), (64, 0, 32, 0), (56, 4, 128, 0), (64, 4, 128, 0)):
        variants.append(("strip%d_rows%d_halo%d%s" % (outw, rows, hy, "_4waves_per_cu" if lds else ""),
                         lambda outw=outw, rows=rows, hy=hy, lds=lds: lib.probe_strip_copy(
                             src.data_ptr(), dst.data_ptr(), L, L, outw, rows, hy, lds, sp)))
    variants.append(("flat_float4", lambda: lib.probe_flat_copy(src.data_ptr(), dst.data_ptr(), n, sp)))
    # the strip-blocked layout f[block][row][k][56] on 110 blocks (6160 columns)
    # x L rows: same node count within 0.3%; GB/s scaled to its own bytes below
    nb = (L + 55) // 56
    for hy, rows, lds in ((4, 32, 0), (4, 32, 36864), (4, 64, 36864), (0, 32, 36864)):
        variants.append(("blocked56_rows%d_halo%d%s" % (rows, hy, "_4waves_per_cu" if lds else ""),
                         lambda hy=hy, rows=rows, lds=lds: lib.probe_blocked_copy(
                             src.data_ptr(), dst.data_ptr(), nb, L, rows, hy, lds, sp)))
    out = {}
    for name, fn in variants:
        rc = fn()
        if rc != 0:
            raise RuntimeError("probe %s failed: hip error %d" % (name, rc))
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        times.sort()
        b = 2.0 * 4 * nblk if name.startswith("blocked") else algo
        out[name] = {"best_ms": round(times[0], 4), "median_ms": round(times[len(times) // 2], 4),
                     "GBs_best": round(b / (times[0] * 1e-3) / 1e9, 1),
                     "GBs_median": round(b / (times[len(times) // 2] * 1e-3) / 1e9, 1)}
        print("[copy-probe] %-34s best %.4f ms (%.0f GB/s), median %.4f ms (%.0f GB/s)"
              % (name, times[0], out[name]["GBs_best"], times[len(times) // 2], out[name]["GBs_median"]),
              file=sys.stderr, flush=True)
    ok = bool(torch.equal(src[:nblk], dst[:nblk]))
    del src, dst
    torch.cuda.empty_cache()
    return {"metric": "copy ceilings of the step's access shape", "unit": "GB/s (algorithmic bytes)",
            "bytes_per_launch": algo, "lattice": [L, L], "planes": 16, "dtype": "f32", "reps": reps,
            "last_copy_matches_source": ok, "variants": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--L", type=int, default=6144)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-only", action="store_true")
    ap.add_argument("--launch", default=None,
                    help="fixed launch shape ROWS,WAVES (rows per strip and workgroup; wavefronts per workgroup, "
                         "or 0 for a pair of wavefronts per strip) of the FP32 stepper instead of the autotuner's")
    ap.add_argument("--launch64", default=None, help="the same for the FP64 stepper (WAVES at most 2)")
    ap.add_argument("--error-steps", type=int, default=0,
                    help="step both steppers on to this many steps after the timing before comparing them "
                         "(error_fp32dev; e.g. 5000, the workload's run length)")
    ap.add_argument("--regularize", action="store_true",
                    help="regularized collision (Eq. ereg) instead of plain BGK; not the headline")
    ap.add_argument("--scheme", type=int, default=2, choices=(1, 2),
                    help="advection scheme: 2 = CTU2 (the headline), 1 = CTU1")
    ap.add_argument("--batched", action="store_true",
                    help="instead of the 6144^2 lattice: the 32-run sweep of uneven lattices in one batched, "
                         "graph-captured launch per step against the same runs stepped one after another")
    ap.add_argument("--batched-tail", action="store_true",
                    help="instead of the 6144^2 lattice: the 32-run sweep held 1, 2 and 4 times over in one batch, "
                         "splitting the batched step's time into a part that grows with the work and a fixed part "
                         "(launch and tail)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="instead of the stepper: plain copies of the FP32 field in the step's access shape and "
                         "simpler ones (memory-side ceilings, GB/s of algorithmic bytes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy 5 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the stepper runs on one GPU only (the lattice is advanced on a single device; "
              "--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1802_01272_amd import inputs as I
    from paper_1802_01272_amd import lbm

    torch.cuda.set_device(0)
    if args.batched:
        print(json.dumps(batched_sweep(args, torch, I, lbm)), flush=True)
        return
    if args.batched_tail:
        print(json.dumps(batched_tail(args, torch, I, lbm)), flush=True)
        return
    if args.copy_probe:
        print(json.dumps(copy_probe(args, torch)), flush=True)
        return
    if args.copy_calibration:
        src_t = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst_t = torch.empty_like(src_t)
        for _ in range(5):
            dst_t.copy_(src_t)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 5 copies of %d bytes" % (src_t.numel() * 4), file=sys.stderr, flush=True)
        del src_t, dst_t
    fixed = {"f32": tuple(int(v) for v in args.launch.split(",")) if args.launch else None,
             "f64": tuple(int(v) for v in args.launch64.split(",")) if args.launch64 else None}
    w = I.large_lattice(args.L)
    w.regularize = 1 if args.regularize else 0
    w.scheme = args.scheme
    rho, ux, uy = w.fields()
    nodes = w.Lx * w.Ly
    results = {}
    runs = {}
    for name, prec in (("f32", lbm.FP32_DEV), ("f64", lbm.FP64)):
        if name == "f64" and args.fp32_only:
            continue
        p = lbm.Params.from_workload(w, precision=prec)
        launch = fixed[name] if fixed[name] else (None if args.no_autotune else lbm.autotune(p, steps_per_trial=10))
        run = lbm.Run(p, rho, ux, uy)
        if launch:
            run.set_launch(*launch)
        run.step(args.warmup)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        run.step(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        per = ms / args.steps
        results[name] = {"ms_per_step": per, "mlups": nodes / (per * 1e-3) / 1e6, "wall_s": wall,
                         "launch": run.get_launch()}
        print("[bench] %s: %.4f ms/step, %.1f MLUPS, launch %s" % (name, per, results[name]["mlups"],
                                                                   results[name]["launch"]),
              file=sys.stderr, flush=True)
        runs[name] = run

    # error of the FP32-deviation storage against the FP64 stepper after the same steps
    err = None
    if "f64" in runs:
        done = args.warmup + args.steps
        if args.error_steps > done:
            # both steppers on to the requested step count (after the timing)
            for r in runs.values():
                r.step(args.error_steps - done)
            done = args.error_steps
        r32, x32, y32 = runs["f32"].moments_device()
        r64, x64, y64 = runs["f64"].moments_device()
        umax = torch.sqrt(x64 ** 2 + y64 ** 2).max().clamp_min(1e-300)
        du = torch.sqrt((x32 - x64) ** 2 + (y32 - y64) ** 2)
        drho = ((r32 - r64).abs() / r64.abs())
        err = {"rho_max_rel": float(drho.max()), "rho_rms_rel": float(drho.pow(2).mean().sqrt()),
               "u_max_rel": float(du.max() / umax), "u_rms_rel": float(du.pow(2).mean().sqrt() / umax),
               "steps": done, "against": "FP64 GPU stepper, same input"}
        del r32, x32, y32, r64, x64, y64

    f32 = results["f32"]
    achieved = BYTES_PER_LUP["f32"] * nodes / (f32["ms_per_step"] * 1e-3) / 1e9
    line = {
        "metric": "MLUPS + % HBM roofline, FP32-deviation vs FP64 stepper at stated rho/u error",
        "value": round(f32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "Lx": w.Lx, "Ly": w.Ly, "T_over_Tc": w.T, "rho_ext": round(w.rho_ext, 6),
                   "bubble_radius": w.radius, "tau": w.tau, "kappa": w.kappa, "scheme": "CTU%d" % w.scheme,
                   "regularize": w.regularize,
                   "storage": "FP32 f - w rho_ref", "rho_ref": round(w.rho_ref, 6), "launch": list(f32["launch"])},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic("step_fp32dev_ctu%d%s_%d" % (w.scheme, "_reg" if w.regularize else "", w.Lx),
                                                 f32["launch"])},
    }
    # the second bound of the same kernel: VALU issue (one wavefront
    # instruction per SIMD every 4 cycles, 1024 SIMDs at 2.4 GHz)
    valu = measured_valu("step_fp32dev_ctu%d%s_%d" % (w.scheme, "_reg" if w.regularize else "", w.Lx), f32["launch"])
    if valu:
        ceiling_ms = valu * 4 / (VALU_SIMDS * CLOCK_HZ) * 1e3
        line["valu_bound"] = {"instructions_per_launch": valu, "ceiling_ms": round(ceiling_ms, 4),
                              "frac": round(ceiling_ms / f32["ms_per_step"], 4)}
    if "f64" in results:
        f64 = results["f64"]
        ach64 = BYTES_PER_LUP["f64"] * nodes / (f64["ms_per_step"] * 1e-3) / 1e9
        line["fp64"] = {"mlups": round(f64["mlups"], 1), "ms_per_step": round(f64["ms_per_step"], 5),
                        "achieved_GBs": round(ach64, 1), "frac": round(ach64 / PEAK_HBM_GBS, 4),
                        "launch": list(f64["launch"]),
                        "traffic": measured_traffic("step_fp64_ctu%d%s_%d" % (w.scheme, "_reg" if w.regularize else "", w.Lx),
                                                    f64["launch"])}
        line["speedup_fp32dev_over_fp64"] = round(f64["ms_per_step"] / f32["ms_per_step"], 3)
    if err:
        line["error_fp32dev"] = err
    for r in runs.values():
        r.close()
    del runs
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, rho, ux, uy)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
