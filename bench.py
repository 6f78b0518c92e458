"""Benchmark: fine cells/s per MRCM-OS solve on one MI355X.

One step = one full MRCM-OS solve through the C ABI (Algorithm 1 Steps 1-7:
local factorisations and seed solves, particular solves, interface system
assembly and solve, MRCM-O assembly, N_s smoothing sweeps, pressure and flux
written to device buffers), with the permeability already resident in HBM.

Workload (default): 256 x 256 cells, 16 x 16 subdomains of 16 x 16 cells,
piecewise-linear interface spaces, Gaussian log K (sigma^2 = 4, correlation
0.05), quarter five-spot wells with no-flow boundaries, alpha = 1, five
smoothing steps, overlap 4 (overlaps 0 and 2 are reported beside it).  The
headline value is the FP32-factor + FP64-refinement form; the FP64 form is
timed on the same workload and reported beside it, and the FP32+refinement
flux is compared with the CPU FP64 oracle.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the CPU baseline (oracle) runs single-threaded
for _v in ("OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "OMP_NUM_THREADS"):
    os.environ[_v] = "1"

PEAK_FP64 = 78.6e12  # MI355X dense FP64 (vector and matrix), FLOP/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--overlap", type=int, default=4)
    ap.add_argument("--precision", default="fp32_refine", choices=["fp64", "fp32_refine"])
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other overlaps")
    return ap.parse_args()


def time_solves(wl, precision, steps, warmup, tol):
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    api.configure(ctx, wl, precision, tol=tol, max_refine=30)
    p = torch.empty(wl.ncells, dtype=torch.float64, device="cuda")
    fl = torch.empty(wl.ncells * 2 * wl.dim, dtype=torch.float64, device="cuda")

    def step():
        m.build_basis(ctx)
        m.solve_interface(ctx)
        m.smooth(ctx, wl.nsmooth)
        m.get_pressure(ctx, p)
        m.get_flux(ctx, fl)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    keys = ("ms_basis", "ms_interface", "ms_smooth", "ms_interface_solve")
    phases = {k: 0.0 for k in keys}
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # phase times of separate solves (get_stats synchronises, so it stays
    # out of the timed loop)
    for _ in range(min(steps, 5)):
        step()
        st = m.get_stats(ctx)
        for k in keys:
            phases[k] += st[k] / min(steps, 5)
    st = m.get_stats(ctx)
    m.destroy(ctx)
    return dt, phases, st, p.cpu().numpy(), fl.cpu().numpy()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this MRCM-OS path has no multi-GPU form "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    from inputs import make_workload
    wl = make_workload(args.workload, overlap=args.overlap)
    dt, phases, st, p, fl = time_solves(wl, args.precision, args.steps, args.warmup, args.tol)
    other = "fp64" if args.precision == "fp32_refine" else "fp32_refine"
    dt2, ph2, st2, _, _ = time_solves(wl, other, max(3, args.steps // 2), 2, args.tol)
    extra = {}
    if not args.no_extra and args.workload == "c2":
        for l in (0, 2, 4):
            if l == args.overlap:
                continue
            w2 = make_workload(args.workload, overlap=l)
            d3, ph3, _, _, _ = time_solves(w2, args.precision, max(3, args.steps // 2), 2, args.tol)
            extra["overlap_%d" % l] = {"ms_per_step": round(d3 * 1e3, 4), "value": w2.ncells / d3,
                                       **{k: round(v, 4) for k, v in ph3.items()}}
    # interface factor + solve: algorithmic flops of the banded LU with
    # partial pivoting (2 kl (kl+ku) per column) and of the triangular solves
    n, kl, ku = st["n_unknowns"], st["band_kl"], st["band_ku"]
    flops = 2.0 * n * kl * (kl + ku) + 2.0 * n * (2 * kl + ku)
    ms_lu = phases["ms_interface_solve"]
    achieved = flops / (ms_lu * 1e-3) if ms_lu > 0 else 0.0
    line = {
        "metric": "fine cells/s per MRCM-OS solve, FP32+refine vs FP64, at flux err <=1e-6",
        "value": wl.ncells / dt,
        "unit": "fine cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32_refine" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %dx%d cells, subdomains %s, overlap %d, %s spaces, %d smoothing steps"
                   % (args.workload, wl.ncell[0], wl.ncell[1], "x".join(map(str, wl.sub)),
                      wl.overlap, wl.space, wl.nsmooth),
                   "precision": args.precision, "interface_unknowns": n,
                   "band_kl": kl, "band_ku": ku},
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "refine": {"max_fp32_solves": st["refine_max_iters"],
                   "max_backward_error": st["refine_max_resid"]},
        other: {"value": wl.ncells / dt2, "ms_per_step": dt2 * 1e3,
                "phases_ms": {k: round(v, 4) for k, v in ph2.items()}},
        "other_overlaps": extra,
        "roofline": {"kernel": "k_bandlu_blocked (interface LU, one workgroup)", "bound": "alu",
                     "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64, "traffic": None},
    }
    if not args.no_cpu_baseline:
        from oracle import mrcm as oracle_mrcm
        times = []
        ref = None
        for _ in range(3):
            t = time.perf_counter()
            ref = oracle_mrcm.solve(wl)
            times.append(time.perf_counter() - t)
        tcpu = float(np.median(times))
        line["cpu_baseline"] = {"value": wl.ncells / tcpu, "unit": "fine cells/s", "cores": 1,
                                "kind": "oracle",
                                "sample": "median of 3 full oracle solves of the benchmark workload "
                                          "(%.2f s each, one thread)" % tcpu}
        rp, rf = ref.pressure(), ref.flux().ravel()
        line["err_vs_oracle"] = {
            "flux_rel_l2": float(np.linalg.norm(fl - rf) / np.linalg.norm(rf)),
            "pressure_rel_l2": float(np.linalg.norm(p - rp) / np.linalg.norm(rp))}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
