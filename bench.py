#!/usr/bin/env python3
"""Benchmark of the compact 8th-order gas-kinetic scheme on one MI355X.

A step is one two-stage MSMD step of the whole hot path (reconstruction,
WENO-Z, interface distribution at every Gauss point of every face, MSMD
update of averages and gradients) over the 2-D Navier-Stokes workload:
isentropic vortex (strength 5) plus a seeded random-phase acoustic
perturbation (amplitude 1e-3, wavenumbers 1..32), mu = 1e-4, periodic
[0, 10]^2, 1024 x 1024 cells, CFL 0.3.  Inputs are synthetic and resident in
HBM before the timed region.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per MSMD step, 2D 8th-order GKS: FP32-mixed vs FP64 at equal L1"
FP64_VALU_PEAK = 78.6  # TFLOP/s, MI355X vector FP64
FP32_VALU_PEAK = 157.3


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024, help="cells per direction")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-window", type=int, default=400, help="oracle sample: window edge in cells, one step")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run one device-to-device copy of this many MiB (calibrates FETCH_SIZE/WRITE_SIZE)")
    return ap.parse_args()


def cpu_baseline(prob, dt, window):
    """The oracle advancing a window of the same initial data (extrapolated
    edges) by one MSMD step with the GPU's first dt."""
    import numpy as np
    import oracle

    n = prob.nx
    w = min(window, n)
    j0 = (n - w) // 2
    sl = (slice(j0, j0 + w), slice(j0, j0 + w))
    W, Wx, Wy = (np.ascontiguousarray(a[sl]) for a in (prob.W, prob.Wx, prob.Wy))
    dx = (prob.xhi - prob.xlo) / n
    kw = prob.oracle_kwargs()
    kw.update(xlo=0.0, xhi=w * dx, ylo=0.0, yhi=w * dx, bc=(1, 1, 1, 1), dt_fixed=dt, t_end=dt)
    t0 = time.perf_counter()
    oracle.run(2, W, Wx, Wy, **kw)
    el = time.perf_counter() - t0
    return {"value": w * w / el, "unit": "cell-updates/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"one MSMD step on the central {w}x{w} window of the same {n}x{n} initial data "
                      f"(extrapolated window edges, dt of the first GPU step), {el:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (the scheme's single-GPU path); "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
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

    from paper_1901_00261_amd import gks
    from paper_1901_00261_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    prob = wl.isentropic_vortex_2d(args.n, mu=1e-4, eps=5.0, acoustic_amp=1e-3, nmodes=32, seed=3,
                                   order=8, recon=1, cfl=0.3, t_end=1e9)
    # inputs resident in HBM (torch owns them), handed to the library by device pointer
    tW, tWx, tWy = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (prob.W, prob.Wx, prob.Wy))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream
    prec = gks.PREC_FP64 if args.precision == "fp64" else gks.PREC_FP32_MIXED
    S = gks.Solver(prob, prec, stream=stream, device_arrays=[(tW.data_ptr(), tWx.data_ptr(), tWy.data_ptr())])
    del tW, tWx, tWy
    if args.warmup:
        S.step(args.warmup)
    t_before = S.state(0)[3]
    S.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    W, _, _, t_after, nsteps = S.state(0)
    flux_ms, flux_n = S.kernel_time(gks.KERNEL_FLUX)
    row_ms, row_n = S.kernel_time(gks.KERNEL_ROW)
    cell_ms, cell_n = S.kernel_time(gks.KERNEL_CELL)
    S.close()
    cells = prob.nx * prob.ny
    value = cells * args.steps / el

    # roofline of the dominant kernel (Gauss-point interface kernel):
    # algorithmic flops per launch = face rows per launch * 3 Gauss points *
    # flops per Gauss point (operation count of the interface arithmetic)
    ops = json.load(open(os.path.join(ROOT, "paper_1901_00261_amd", "opcount.json")))
    fpg = ops["gauss_point_ns"]["flops"]
    rows_per_launch = ((prob.nx + 1) * prob.ny + (prob.ny + 1) * prob.nx) / 2.0
    flops_per_launch = rows_per_launch * 3 * fpg
    avg_s = flux_ms / max(flux_n, 1) / 1e3
    achieved = flops_per_launch / avg_s / 1e12
    peak = FP64_VALU_PEAK
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64acc",
        "data": "synthetic",
        "config": {"workload": f"2-D Navier-Stokes isentropic vortex + seeded acoustic perturbation, "
                               f"{prob.nx}x{prob.ny} periodic on [0,10]^2, 8th-order compact WENO-Z GKS, "
                               f"mu=1e-4, CFL 0.3",
                   "nx": prob.nx, "ny": prob.ny, "precision": args.precision, "t_reached": t_after,
                   "kernel_ms_per_step": {"interface": flux_ms / args.steps, "face_row": row_ms / args.steps,
                                          "cell_update": cell_ms / args.steps}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "gp2d_kernel (interface, Gauss points)",
                     "avg_launch_ms": avg_s * 1e3, "launches": flux_n},
    }
    ok = bool(np.isfinite(W).all()) and nsteps == args.warmup + args.steps and t_after > t_before
    if not ok:
        line["error"] = "non-finite state or missing steps"
    if not args.no_cpu_baseline:
        dt0 = (t_after - t_before) / args.steps
        line["cpu_baseline"] = cpu_baseline(prob, dt0, args.cpu_window)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
