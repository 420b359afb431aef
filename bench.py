#!/usr/bin/env python3
"""Benchmark of the compact 8th-order gas-kinetic scheme on one MI355X.

Default line: a step is one two-stage MSMD step of the whole hot path
(face-row reconstruction with WENO-Z, tangential reconstruction and the
interface distribution at every Gauss point of every face, MSMD update of
averages and gradients) over the 2-D Navier-Stokes workload: isentropic
vortex (strength 5) plus a seeded random-phase acoustic perturbation
(amplitude 1e-3, wavenumbers 1..32), mu = 1e-4, periodic [0, 10]^2,
1024 x 1024 cells, CFL 0.3.  FP64 gives `value`; the FP32-mixed form is
timed on the same input and reported beside it.  Inputs are synthetic and
resident in HBM before the timed region.  Prints one JSON line.

Other modes (reports, not the headline line):
  --workload batch1d    256 uneven 1-D Riemann problems run to t = 0.14
  --workload riemann2d  2-D four-quadrant Euler Riemann problem, 4096^2
  --study equal-l1      L1(rho) and throughput of both precisions over
                        N = 128..1024 against an FP64 2048^2 reference
                        (the vortex, or with --workload riemann2d the
                        four-quadrant problem)
  --workload cpu-configs  the oracle's rates on bounded samples of each
                        workload, all host threads and one (no GPU)
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per MSMD step, 2D 8th-order GKS: FP32-mixed vs FP64 at equal L1"
# MI355X vector peaks: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz = 78.6
# TFLOP/s for FP64 and unpacked FP32; 157.3 TFLOP/s is the packed-FP32 peak.
FP64_VALU_PEAK = 78.6
FP32_VALU_PEAK = 157.3
HBM_PEAK = 8000.0  # GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gp2d_hbm_traffic_vortex1024.md")
VALU_FILE = os.path.join(ROOT, "profiles", "gp2d_valu_counters_vortex1024.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1901_00261_amd", "csrc", f)
                  for f in ("gks_math.h", "gks_kernels.h", "gks_api.hip")]


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=0, help="cells per direction (2-D workloads)")
    ap.add_argument("--workload", choices=["vortex2d", "batch1d", "riemann2d", "cpu-configs"], default="vortex2d",
                    help="cpu-configs: the CPU-baseline leg (the oracle) on bounded samples of each workload (no GPU)")
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--study", choices=["none", "equal-l1"], default="none")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-window", type=int, default=400, help="oracle sample: window edge in cells, one step")
    ap.add_argument("--cpu-window1", type=int, default=100, help="oracle sample on one thread: window edge")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run one device-to-device copy of this many MiB (calibrates FETCH_SIZE/WRITE_SIZE)")
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _counter_summary(path, prec):
    """The machine-readable block of a committed rocprofv3 counter summary,
    entry for precision prec (0 FP64, 1 FP32-mixed), or None when the file
    is absent or the kernel sources changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), flags=re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("fp64" if prec == 0 else "mixed")


def measured_traffic(prec):
    """HBM bytes per launch of the interface kernel (FETCH_SIZE and
    WRITE_SIZE, scaled by a device copy of known size)."""
    return _counter_summary(TRAFFIC_FILE, prec)


def valu_peak(prec):
    """Vector peak for the interface kernel's executed operation mix: a
    launch that executes F64 FP64 and F32 FP32 flops needs at least
    F64/78.6 + F32/157.3 (TFLOP/s) of time, so its peak is their sum over
    that.  FP64 counts against 78.6 alone; without the counters, FP32-mixed
    counts against 157.3 (an upper bound)."""
    if prec == 0:
        return FP64_VALU_PEAK, "fp64 vector"
    d = _counter_summary(VALU_FILE, prec)
    if not d:
        return FP32_VALU_PEAK, "fp32 vector (no operation-mix counters for these sources)"
    f64, f32 = d["f64_flops_per_launch"], d["f32_flops_per_launch"]
    peak = (f64 + f32) / (f64 / FP64_VALU_PEAK + f32 / FP32_VALU_PEAK)
    return peak, f"executed mix {f32 / (f64 + f32):.2f} FP32 / {f64 / (f64 + f32):.2f} FP64 of 157.3 / 78.6"


def vortex(n):
    from paper_1901_00261_amd import workloads as wl
    return wl.isentropic_vortex_2d(n, mu=1e-4, eps=5.0, acoustic_amp=1e-3, nmodes=32, seed=3,
                                   order=8, recon=1, cfl=0.3, t_end=1e9)


def device_solver(prob, prec):
    """Inputs moved to HBM as torch tensors and handed to the library by
    device pointer; the library runs on torch's current stream."""
    import numpy as np
    import torch
    from paper_1901_00261_amd import gks
    dev = torch.device("cuda:0")
    ts = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (prob.W, prob.Wx, prob.Wy)]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream
    S = gks.Solver(prob, prec, stream=stream, device_arrays=[tuple(t.data_ptr() for t in ts)])
    torch.cuda.synchronize()
    del ts
    return S


def time_2d(prob, prec, steps, warmup):
    """Warm-up, then `steps` MSMD steps timed end to end as the library runs
    them (graph replays on the library's stream, torch's current stream).  A
    second run over the same steps, from the same initial data, records HIP
    events around every kernel launch for the per-kernel times (event timing
    issues the launches one by one, without the graph)."""
    import numpy as np
    import torch
    from paper_1901_00261_amd import gks
    out = {}
    for timing in (False, True):
        S = device_solver(prob, prec)
        if warmup:
            S.step(warmup)
        t_before = S.state(0)[3]
        if timing:
            S.timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        W, _, _, t_after, nsteps = S.state(0)
        ok = bool(np.isfinite(W).all()) and nsteps == warmup + steps and t_after > t_before
        if not timing:
            out.update(elapsed=el, ok=ok, t_before=t_before, t_after=t_after)
        else:
            out["elapsed_events"] = el
            out["ok"] = out["ok"] and ok
            out["kernels"] = {name: S.kernel_time(kid) for name, kid in
                              (("interface", gks.KERNEL_FLUX), ("face_row", gks.KERNEL_ROW),
                               ("cell_update", gks.KERNEL_CELL))}
        S.close()
    return out


def roofline_2d(prob, res, ops, prec):
    """Interface (Gauss-point) kernel: algorithmic flops per launch = face
    rows per launch x 3 Gauss points x flops per Gauss point (stage 1 and
    stage 2 launches alternate, so the mean of the two stage counts).  A
    direction with n cells has n + 1 distinct faces, n when periodic (its
    last face is its first)."""
    key = "gauss_point_ns" if prob.mu > 0 else "gauss_point_euler"
    fpg = 0.5 * (ops[key]["flops"] + ops[key + "_s2"]["flops"])
    nfx = prob.nx + (0 if prob.bc[0] == 0 else 1)
    nfy = prob.ny + (0 if prob.bc[2] == 0 else 1)
    rows = (nfx * prob.ny + nfy * prob.nx) / 2.0
    flops = rows * 3 * fpg
    ms, n = res["kernels"]["interface"]
    avg_s = ms / max(n, 1) / 1e3
    achieved = flops / avg_s / 1e12
    peak, basis = valu_peak(prec)
    out = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
           "traffic": None, "kernel": "gp2d_kernel (interface, Gauss points)", "avg_launch_ms": avg_s * 1e3,
           "launches": n, "flops_per_launch": flops, "flops_per_gauss_point": fpg, "peak_basis": basis}
    traffic = measured_traffic(prec) if (prob.nx, prob.ny, prob.mu > 0) == (1024, 1024, True) else None
    if traffic:
        out["traffic"] = traffic["bytes_per_launch"]
        out["traffic_GBps"] = traffic["bytes_per_launch"] / avg_s / 1e9
        out["algorithmic_bytes_per_launch"] = traffic["algorithmic_bytes_per_launch"]
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, dt, window, window1):
    """The oracle advancing a window of the same initial data (extrapolated
    edges) by one MSMD step with the GPU's dt, on all host threads (the
    reported baseline) and on one thread (a smaller window)."""
    import numpy as np
    import oracle

    def one(w, threads):
        n = prob.nx
        w = min(w, n)
        j0 = (n - w) // 2
        sl = (slice(j0, j0 + w), slice(j0, j0 + w))
        W, Wx, Wy = (np.ascontiguousarray(a[sl]) for a in (prob.W, prob.Wx, prob.Wy))
        dx = (prob.xhi - prob.xlo) / n
        kw = prob.oracle_kwargs()
        kw.update(xlo=0.0, xhi=w * dx, ylo=0.0, yhi=w * dx, bc=(1, 1, 1, 1), dt_fixed=dt, t_end=dt)
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        oracle.run(2, W, Wx, Wy, **kw)
        el = time.perf_counter() - t0
        return w * w / el, el, w

    nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    v, el, w = one(window, nthreads)
    v1, el1, w1 = one(window1, 1)
    oracle.set_threads(nthreads)
    return {"value": v, "unit": "cell-updates/s", "cores": nthreads, "kind": "oracle",
            "sample": f"one MSMD step on the central {w}x{w} window of the same {prob.nx}x{prob.ny} initial data "
                      f"(extrapolated window edges, dt of the GPU steps), {el:.1f} s on {nthreads} threads",
            "cpu_model": cpu_model(),
            "single_thread": {"value": v1, "unit": "cell-updates/s", "cores": 1,
                              "sample": f"one MSMD step on the central {w1}x{w1} window, {el1:.1f} s"}}


# Algorithmic HBM bytes of one 2-D MSMD step per cell: W, W_x, W_y (12
# doubles) read and written in each stage plus the FP64 partials written in
# stage 1 and read in stage 2 -- 72 doubles (both precisions keep the state
# and the partials in FP64).
STEP_BYTES_2D = 576


def hbm_step(value):
    """Step-level HBM roof: algorithmic bytes per cell-update times the
    measured cell-updates/s, against the 8 TB/s peak."""
    gbps = value * STEP_BYTES_2D / 1e9
    return {"bytes_per_cell_update": STEP_BYTES_2D, "achieved_GBps": gbps, "peak_GBps": HBM_PEAK,
            "frac": gbps / HBM_PEAK}


def step_roof(value, ops, prec, mu):
    """Step-level roofline: T_bound = max(B_alg / 8 TB/s, F_alg / vector
    peak) per cell-update against the measured time per cell-update, with
    F_alg = 2 directions x (2 stages x face row + 3 Gauss points x (stage-1
    + stage-2 point)) from the operation counts (the cell update's ~100
    flops left out) and the vector peak of the precision's executed mix."""
    key = "gauss_point_ns" if mu > 0 else "gauss_point_euler"
    f_alg = 2 * (2 * ops["face_row_2d"]["flops"] + 3 * (ops[key]["flops"] + ops[key + "_s2"]["flops"]))
    peak, basis = valu_peak(prec)
    t_alu = f_alg / (peak * 1e12)
    t_hbm = STEP_BYTES_2D / (HBM_PEAK * 1e9)
    t_meas = 1.0 / value
    return {"flops_per_cell_update": f_alg, "bytes_per_cell_update": STEP_BYTES_2D, "peak_TFLOPs": peak,
            "peak_basis": basis, "t_bound_ns": max(t_alu, t_hbm) * 1e9, "t_meas_ns": t_meas * 1e9,
            "bound": "alu" if t_alu >= t_hbm else "hbm", "frac": max(t_alu, t_hbm) / t_meas}


def load_ops():
    return json.load(open(os.path.join(ROOT, "paper_1901_00261_amd", "opcount.json")))


def bench_vortex(args):
    n = args.n or 1024
    prob = vortex(n)
    ops = load_ops()
    precs = {"fp64": [0], "mixed": [1], "both": [0, 1]}[args.precision]
    results = {p: time_2d(prob, p, args.steps, args.warmup) for p in precs}
    main_p = precs[0]
    res = results[main_p]
    cells = prob.nx * prob.ny
    value = cells * args.steps / res["elapsed"]
    roof = roofline_2d(prob, res, ops, main_p)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_p == 0 else "f32+f64acc",
        "data": "synthetic",
        "config": {"workload": f"2-D Navier-Stokes isentropic vortex (strength 5) + seeded acoustic perturbation "
                               f"(1e-3, k=1..32), {prob.nx}x{prob.ny} periodic on [0,10]^2, 8th-order compact "
                               f"WENO-Z GKS, mu=1e-4, CFL 0.3",
                   "nx": prob.nx, "ny": prob.ny, "precision": "fp64" if main_p == 0 else "mixed",
                   "t_reached": res["t_after"],
                   "kernel_ms_per_step": {k: v[0] / args.steps for k, v in res["kernels"].items()},
                   "ms_per_step_with_kernel_events": res["elapsed_events"] / args.steps * 1e3},
        "roofline": roof,
        "hbm_step": hbm_step(value),
        "step_roof": step_roof(value, ops, main_p, prob.mu),
    }
    if 1 in results and main_p == 0:
        rm = results[1]
        vm = cells * args.steps / rm["elapsed"]
        line["config"]["mixed"] = {
            "value": vm, "ms_per_step": rm["elapsed"] / args.steps * 1e3, "speedup_vs_fp64": vm / value,
            "hbm_step": hbm_step(vm),
            "step_roof": step_roof(vm, ops, 1, prob.mu),
            "kernel_ms_per_step": {k: v[0] / args.steps for k, v in rm["kernels"].items()},
            "ms_per_step_with_kernel_events": rm["elapsed_events"] / args.steps * 1e3,
            "roofline": roofline_2d(prob, rm, ops, 1)}
    if not all(r["ok"] for r in results.values()):
        line["error"] = "non-finite state or missing steps"
    if not args.no_cpu_baseline:
        dt0 = (res["t_after"] - res["t_before"]) / args.steps
        line["cpu_baseline"] = cpu_baseline(prob, dt0, args.cpu_window, args.cpu_window1)
    return line


def bench_riemann2d(args):
    from paper_1901_00261_amd import workloads as wl
    n = args.n or 4096
    prob = wl.riemann_2d(n, seed=5, order=8, recon=1, cfl=0.3)
    ops = load_ops()
    precs = {"fp64": [0], "mixed": [1], "both": [0, 1]}[args.precision]
    out = {"workload": f"2-D Euler four-quadrant Riemann problem, {n}x{n} on [0,1]^2, seeded quadrant states "
                       f"(seed 5), 8th-order compact WENO-Z, CFL 0.3, extrapolated boundaries",
           "steps": args.steps, "warmup": args.warmup, "unit": "cell-updates/s"}
    for p in precs:
        r = time_2d(prob, p, args.steps, args.warmup)
        out["fp64" if p == 0 else "mixed"] = {
            "value": n * n * args.steps / r["elapsed"], "ms_per_step": r["elapsed"] / args.steps * 1e3, "ok": r["ok"],
            "t_reached": r["t_after"], "kernel_ms_per_step": {k: v[0] / args.steps for k, v in r["kernels"].items()},
            "roofline": roofline_2d(prob, r, ops, p),
            "step_roof": step_roof(n * n * args.steps / r["elapsed"], ops, p, prob.mu)}
    return out


def bench_batch1d(args):
    """All 256 problems to t = 0.14 (graph-replayed steps, autotuned launch);
    value = sum over problems of cells x steps / wall time.  A second run
    with kernel events gives the stage-kernel durations."""
    import numpy as np
    import torch
    from paper_1901_00261_amd import gks
    from paper_1901_00261_amd import workloads as wl
    probs = wl.batch_1d()
    ops = load_ops()
    precs = {"fp64": [0], "mixed": [1], "both": [0, 1]}[args.precision]
    out = {"workload": "batched 1-D Euler Riemann problems: 256 problems, N ~ U[200,4000] (seed 4), order 6 or 8, "
                       "WENO-Z, CFL 0.3, t = 0.14, extrapolated boundaries", "unit": "cell-updates/s"}
    for p in precs:
        rec = {}
        for timing in (False, True):
            S = gks.Solver(probs, p)
            # autotune + first step (untimed); a problem that meets a non-physical
            # state stops there and is listed below, the others go on
            S.step(1, raise_on_error=False)
            if timing:
                S.timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            upd = 0
            steps = 0
            while True:
                r = S.step(128, raise_on_error=False)
                upd += S.cell_updates()
                steps += 128
                if r == 0:
                    break
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            stopped = [k for k in range(len(probs)) if S.status(k) == gks.GKS_ENONPHYS]
            if not timing:
                rec.update(value=upd / el, seconds=el, cell_updates=upd, launch=S.launch_config(),
                           stopped_nonphysical=stopped)
            else:
                ms, nl = S.kernel_time(gks.KERNEL_FLUX)
                # the active set shrinks as problems finish, so the figure is the
                # mean over the run: algorithmic flops of all faces (about one per
                # cell-update per stage) over the summed stage-kernel time
                f1 = ops["face_1d"]["flops"] + ops["face_1d_s2"]["flops"]
                achieved = upd * f1 / (ms / 1e3) / 1e12
                # FP32-mixed against the FP32 vector peak: an upper bound (the
                # state, the exponentials and the MSMD sums stay FP64)
                peak = FP64_VALU_PEAK if p == 0 else FP32_VALU_PEAK
                rec["stage_kernels"] = {"ms_total": ms, "launch_pairs": nl, "mean_pair_ms": ms / max(nl, 1),
                                        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                                                     "unit": "TFLOP/s", "frac": achieved / peak}}
            S.close()
        out["fp64" if p == 0 else "mixed"] = rec
    return out


def cpu_baseline_configs(args):
    """The CPU-baseline leg on every workload: the oracle's own rate on
    bounded samples, on all host threads and on one (a reported baseline,
    not the target): the 1-D sine
    (full run), the first problems of the seeded Riemann set (full runs), a
    window of the vortex (one step), problems of the uneven batch (their
    first steps) and the four-quadrant problem at 256^2 (a few steps)."""
    import oracle
    from paper_1901_00261_amd import workloads as wl
    nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)

    def timed(probs, threads, **over):
        oracle.set_threads(threads)
        upd, t0 = 0, time.perf_counter()
        for p in probs:
            r = oracle.run(p.dim, p.W, p.Wx, p.Wy, **{**p.oracle_kwargs(), **over})
            upd += p.nx * (p.ny if p.dim == 2 else 1) * r[4]
        el = time.perf_counter() - t0
        return {"value": upd / el, "cell_updates": upd, "seconds": el, "cores": threads}

    batch = wl.batch_1d()
    legs = {
        "sine 1-D N=80, 6th linear, full run to t=2": (lambda: [wl.sine_wave_1d(80, order=6, recon=0)], {}, {}),
        "Riemann set N=400, 8th WENO-Z, full runs (problems 0-3 / 0)": (
            lambda: wl.riemann_set_1d(4, n=400), {}, {"one": lambda: wl.riemann_set_1d(1, n=400)}),
        "uneven batch, problems 0-7, first 40 steps": (lambda: batch[:8], {"max_steps": 40},
                                                       {"one": lambda: batch[:2]}),
        "four-quadrant Riemann 256^2, 8th WENO-Z, 4 steps / 1 step": (
            lambda: [wl.riemann_2d(256, seed=5, order=8, recon=1, cfl=0.3)], {"max_steps": 4},
            {"over1": {"max_steps": 1}}),
    }
    out = {"cpu_model": cpu_model(), "threads": nthreads, "unit": "cell-updates/s", "legs": {}}
    for name, (mk, over, one) in legs.items():
        rec = {"all_threads": timed(mk(), nthreads, **over)}
        rec["one_thread"] = timed(one.get("one", mk)(), 1, **one.get("over1", over))
        out["legs"][name] = rec
        print(name, json.dumps(rec), file=sys.stderr, flush=True)
    oracle.set_threads(nthreads)
    return out


def study_equal_l1(args):
    """Equal-L1 study: T3 = time reached by 200 FP64 steps at 1024^2;
    reference = FP64 at 2048^2 to T3; for N = 128..1024 and both
    precisions, L1(rho) against the reference block-averaged to N^2 (exact
    cell averages of the reference field) and the measured cell-updates/s
    of the whole run.  Workloads: the smooth Navier-Stokes vortex (default)
    or, with --workload riemann2d, the shock-dominated four-quadrant Euler
    Riemann problem."""
    import numpy as np
    import torch
    from paper_1901_00261_amd import gks
    from paper_1901_00261_amd import workloads as wl
    log = lambda *a: print(*a, file=sys.stderr, flush=True)

    def run_to(prob, prec, t_end=None, steps=None):
        if t_end is not None:
            prob.t_end = t_end
        S = gks.Solver(prob, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if steps is not None:
            S.step(steps)
        else:
            # one eight-step graph replay per call, so that at most seven
            # idle steps follow the step that reaches t_end
            while S.step(8) > 0:
                pass
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        W, _, _, t, n = S.state(0)
        S.close()
        return W, t, n, el

    if args.workload == "riemann2d":
        make = lambda n: wl.riemann_2d(n, seed=5, order=8, recon=1, cfl=0.3)
        name = "2-D Euler four-quadrant Riemann problem (seed 5), [0,1]^2, extrapolated boundaries"
    else:
        make = vortex
        name = "2-D Navier-Stokes vortex + seeded acoustic perturbation, periodic [0,10]^2"
    base = make(1024)
    _, T3, n3, _ = run_to(base, 0, steps=200)
    log(f"T3 = {T3:.9f} after {n3} FP64 steps at 1024^2")
    ref_prob = make(2048)
    Wref, tr, nr, elr = run_to(ref_prob, 0, t_end=T3)
    log(f"reference 2048^2: {nr} steps, t = {tr:.9f}, {elr:.2f} s")
    rho_ref = Wref[:, :, 0]
    rows = []
    for N in (128, 256, 512, 1024):
        prob = base if N == 1024 else make(N)
        f = 2048 // N
        ref_N = rho_ref.reshape(N, f, N, f).mean(axis=(1, 3))
        for prec in (0, 1):
            W, t, n, el = run_to(prob, prec, t_end=T3)
            l1 = float(np.abs(W[:, :, 0] - ref_N).mean())
            linf = float(np.abs(W[:, :, 0] - ref_N).max())
            row = {"N": N, "precision": "fp64" if prec == 0 else "mixed", "steps": n, "t": t, "L1_rho": l1,
                   "Linf_rho": linf, "seconds": el, "cell_updates_per_s": N * N * n / el}
            rows.append(row)
            log(json.dumps(row))
    return {"study": "equal-L1", "workload": name, "T3": T3, "reference": {"N": 2048, "steps": nr, "seconds": elr},
            "rows": rows, "equal_L1_pairs": equal_l1_pairs(rows)}


def equal_l1_pairs(rows):
    """For each mixed run, the FP64 grid with the same L1 (log-log
    interpolation in N over the FP64 runs, whose L1 falls with N) and the
    FP64 time to solution there.  A target within 1e-4 (relative) of the
    coarsest or finest FP64 L1 takes that grid; beyond the range: NaN."""
    import numpy as np
    f64 = [r for r in rows if r["precision"] == "fp64"]
    Ns = np.log([x["N"] for x in f64])
    Ls = np.log([x["L1_rho"] for x in f64])
    ts = np.log([x["seconds"] for x in f64])
    order = np.argsort(Ls)
    pairs = []
    for r in rows:
        if r["precision"] != "mixed":
            continue
        lt = math.log(r["L1_rho"])
        if Ls.min() - 1e-4 <= lt <= Ls.max() + 1e-4:
            ln = float(np.interp(min(max(lt, Ls.min()), Ls.max()), Ls[order], Ns[order]))
            n_eq, t_eq = math.exp(ln), math.exp(float(np.interp(ln, Ns, ts)))
        else:
            n_eq, t_eq = float("nan"), float("nan")
        pairs.append({"mixed_N": r["N"], "mixed_L1": r["L1_rho"], "mixed_seconds": r["seconds"],
                      "fp64_N_at_equal_L1": n_eq, "fp64_seconds_at_equal_L1": t_eq})
    return pairs


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures the single-GPU path only; --gpus must be 1 "
              "(multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "cpu-configs":
        print(json.dumps(cpu_baseline_configs(args)), flush=True)
        return
    import torch

    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8}))
        return
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.study == "equal-l1":
        print(json.dumps(study_equal_l1(args)), flush=True)
    elif args.workload == "vortex2d":
        print(json.dumps(bench_vortex(args)), flush=True)
    elif args.workload == "riemann2d":
        print(json.dumps(bench_riemann2d(args)), flush=True)
    else:
        print(json.dumps(bench_batch1d(args)), flush=True)


if __name__ == "__main__":
    main()
