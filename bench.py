"""Benchmark: fine cells/s per MRCM-OS solve on one MI355X.

One step = one full MRCM-OS solve through the C ABI (Algorithm 1 Steps 1-7:
local factorisations and seed solves, particular solves, interface system
assembly and solve, MRCM-O assembly, N_s smoothing sweeps, pressure and flux
written to device buffers), with the permeability already resident in HBM.

Workload (default): 256 x 256 cells, 16 x 16 subdomains of 16 x 16 cells,
piecewise-linear interface spaces, Gaussian log K (sigma^2 = 4, correlation
0.05), quarter five-spot wells with no-flow boundaries, alpha = 1, five
smoothing steps, overlap 4 (overlaps 0 and 2 are reported beside it).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--overlap", type=int, default=4)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_refine"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other overlaps")
    return ap.parse_args()


def time_solves(wl, precision, steps, warmup):
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    api.configure(ctx, wl, precision)
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
    phases = {"ms_basis": 0.0, "ms_interface": 0.0, "ms_smooth": 0.0}
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        st = m.get_stats(ctx)
        for k in phases:
            phases[k] += st[k]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st = m.get_stats(ctx)
    m.destroy(ctx)
    for k in phases:
        phases[k] /= steps
    return dt, phases, st, p, fl


def cpu_baseline(wl):
    import numpy as np
    from oracle import mrcm as oracle_mrcm
    times = []
    for _ in range(3):
        t = time.perf_counter()
        oracle_mrcm.solve(wl)
        times.append(time.perf_counter() - t)
    t = float(np.median(times))
    return {"value": wl.ncells / t, "unit": "fine cells/s", "cores": 1, "kind": "oracle",
            "sample": "median of 3 full oracle solves of the benchmark workload (%.2f s each)" % t}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the MRCM-OS path here has no multi-GPU form "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from inputs import make_workload
    wl = make_workload(args.workload, overlap=args.overlap)
    dt, phases, st, p, fl = time_solves(wl, args.precision, args.steps, args.warmup)
    extra = {}
    if not args.no_extra and args.workload == "c2":
        for l in (0, 2, 4):
            if l == args.overlap:
                continue
            w2 = make_workload(args.workload, overlap=l)
            d2, ph2, _, _, _ = time_solves(w2, args.precision, max(3, args.steps // 2), 2)
            extra["overlap_%d" % l] = {"ms_per_step": d2 * 1e3, "value": w2.ncells / d2,
                                       **{k: round(v, 4) for k, v in ph2.items()}}
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
        "dtype": "f64" if args.precision == "fp64" else "f32+f64refine",
        "data": "synthetic",
        "config": {"workload": "%s: %dx%d cells, subdomains %s, overlap %d, %s spaces, %d smoothing steps"
                   % (args.workload, wl.ncell[0], wl.ncell[1], "x".join(map(str, wl.sub)),
                      wl.overlap, wl.space, wl.nsmooth),
                   "precision": args.precision, "interface_unknowns": st["n_unknowns"],
                   "band_kl": st["band_kl"], "band_ku": st["band_ku"]},
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "other_overlaps": extra,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
