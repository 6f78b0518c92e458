"""Benchmark: fine cells/s per MRCM-OS solve on one MI355X.

One step = one full MRCM-OS solve through the C ABI (Algorithm 1 Steps 1-7:
local factorisations and seed solves, particular solves, interface system
assembly and solve, MRCM-O assembly, N_s smoothing sweeps, pressure and flux
written to device buffers), with the permeability already resident in HBM.

Workload (default): 256 x 256 cells, 16 x 16 subdomains of 16 x 16 cells,
piecewise-linear interface spaces, Gaussian log K (sigma^2 = 4, correlation
0.05), quarter five-spot wells with no-flow boundaries, alpha = 1, five
smoothing steps, overlap 4 (overlaps 0 and 2 are reported beside it).

Both forms are timed on the same workload: FP32 factors with FP64 iterative
refinement, and FP64.  Each is compared with the CPU FP64 oracle (relative L2
of flux and pressure).  The headline value is the faster form among those
whose flux error is <= 1e-6 (``--precision`` picks one form instead); the
other form is reported beside it.
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

# MI355X published peaks
PEAK_HBM = 8.0e12        # B/s
PEAK_FP64 = 78.6e12      # FLOP/s, vector (= matrix) FP64
PEAK_FP32 = 157.3e12     # FLOP/s, vector FP32
FLUX_TOL = 1e-6

# HBM bytes per launch of the local kernels on the 256 x 256 workload (overlap
# 4), from two rocprofv3 counter passes (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch).  Each counter is scaled by what it reads for a 256 MiB device copy:
# FETCH_SIZE reports half of the bytes read (factor 2.0), WRITE_SIZE all of
# the bytes written (factor 1.0).  A record holds only while the kernel sources
# hash to the value it was taken with; otherwise the traffic is reported null.
TRAFFIC = {
    # kernel: (source files, sha256 prefix, fetch KiB, write KiB, workload)
    "k_smooth_w": (("local_wave.hip",), "78f5ab5cf02d28dd", 3011.9, 158.0, "c2 overlap 4"),
    "k_local_w": (("local_wave.hip",), "78f5ab5cf02d28dd", 10485.2, 26700.0, "c2 overlap 4"),
    "k_smooth32": (("local_wave32.hip",), "6175ad10e30a35af", 2774.6, 162.0, "c2 overlap 4"),
    "k_local32": (("local_wave32.hip",), "6175ad10e30a35af", 10283.9, 23795.0, "c2 overlap 4"),
}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0


def traffic(kern, wl):
    """Measured HBM bytes per launch of ``kern``, or None when no record fits
    this workload or the kernel source changed since the counters were read."""
    import hashlib
    rec = TRAFFIC.get(kern)
    if rec is None or (wl.name, tuple(wl.ncell), wl.overlap) != ("c2", (256, 256), 4):
        return None
    files, digest, fk, wk, _ = rec
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2404_13811_amd", "csrc")
    for f in files + ("wave_common.h", "local_common.h", "mrcm_internal.h", "pivot4.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != digest:
        return None
    return (fk * FETCH_SCALE + wk * WRITE_SCALE) * 1024.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--overlap", type=int, default=4)
    ap.add_argument("--precision", default="best", choices=["best", "fp64", "fp32_refine"])
    ap.add_argument("--tol", type=float, default=1e-12,
                    help="componentwise backward-error tolerance of the refinement")
    ap.add_argument("--smoothing", default="graph", choices=["graph", "persistent"],
                    help="smoothing sweeps as a replayed graph of per-colour launches, or all "
                         "colour phases of a call in one cooperative launch (FP64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other overlaps")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 256 MiB device-to-device copy (counter calibration)")
    return ap.parse_args()


def time_solves(wl, precision, steps, warmup, tol, persistent=False):
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    api.configure(ctx, wl, precision, tol=tol, max_refine=30)
    m.set_smoothing_persistent(ctx, persistent)
    p = torch.empty(wl.ncells, dtype=torch.float64, device="cuda")
    fl = torch.empty(wl.ncells * 2 * wl.dim, dtype=torch.float64, device="cuda")

    def step():
        m.build_basis(ctx)
        m.solve_interface(ctx)
        m.smooth(ctx, wl.nsmooth)
        m.get_solution(ctx, p, fl)

    # the timed solves enqueue kernels only (no phase-timing events)
    m.set_timing(ctx, False)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # back-to-back solves: the device error flags are read once, at the end
    # of the timed loop (mrcm_wait), so the host enqueues the next solve
    # while the GPU runs this one
    m.set_deferred_errors(ctx, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    m.wait(ctx)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    m.set_deferred_errors(ctx, False)
    # one solve at a time: each ends with its own error read-back (a stream
    # synchronisation), so each solve's wall time is its own
    each = []
    for _ in range(steps):
        t1 = time.perf_counter()
        step()
        each.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    dt_sync = sum(each) / steps
    each.sort()
    m.set_timing(ctx, True)
    # phase and kernel times from the library's HIP events (recorded on the
    # context's stream) over separate solves: get_stats synchronises, so it
    # stays out of the timed loop
    keys = ("ms_basis", "ms_basis_kernel", "ms_interface", "ms_interface_solve", "ms_smooth")
    phases = {k: 0.0 for k in keys}
    nrep = min(steps, 5)
    for _ in range(nrep):
        step()
        st = m.get_stats(ctx)
        for k in keys:
            phases[k] += st[k] / nrep
    st = m.get_stats(ctx)
    st["ms_per_solve_synchronous"] = dt_sync * 1e3
    st["ms_synchronous_median_min_max"] = [round(each[len(each) // 2] * 1e3, 4),
                                           round(each[0] * 1e3, 4), round(each[-1] * 1e3, 4)]
    m.destroy(ctx)
    return dt, phases, st, p.cpu().numpy(), fl.cpu().numpy()


def time_adjoint(wl, reps):
    """Forward solve with checkpointing plus mrcm_adjoint (dJ/dlog K of the
    outflow through the +x side plus a misfit at 16 cells) on one member of
    the batch workload; device wall time per call."""
    import numpy as np
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    nx, ny = wl.ncell
    N = nx * ny
    obs = torch.as_tensor(np.arange(0, N, N // 16)[:16], device="cuda")
    fw = torch.zeros(N, 4, dtype=torch.float64, device="cuda")
    fw[torch.arange(nx - 1, N, nx, device="cuda"), 1] = wl.h
    fw = fw.reshape(-1)
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    api.configure(ctx, wl, "fp64")
    m.set_checkpointing(ctx, True)
    grad = torch.empty(N, dtype=torch.float64, device="cuda")
    tf = ta = 0.0
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.build_basis(ctx)
        m.solve_interface(ctx)
        m.smooth(ctx, wl.nsmooth)
        p = m.get_pressure(ctx)
        m.get_flux(ctx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dJdp = torch.zeros_like(p)
        dJdp[obs] = p[obs] - 0.1
        m.adjoint(ctx, dJdp, fw, grad)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r:  # the first call builds the plan and allocates
            tf += (t1 - t0) / reps
            ta += (t2 - t1) / reps
    m.destroy(ctx)
    return {"workload": "c5 member: 256x256 cells, subdomains 16x16, overlap 2, const spaces, 5 smoothing steps",
            "ms_forward_with_checkpoints": round(tf * 1e3, 4), "ms_gradient": round(ta * 1e3, 4),
            "gradient_over_forward": round(ta / tf, 3)}


def time_batch(members, reps):
    """The c5 batch: every member's forward solve (with checkpoints) and
    gradient, one context and one stream per member, deferred errors (no
    call waits for the device; one mrcm_wait per member ends the batch).
    Device wall time per batch, inputs resident."""
    import numpy as np
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    from inputs import make_workload
    wls = [make_workload("c5", member=k) for k in range(members)]
    nx, ny = wls[0].ncell
    N = nx * ny
    obs = torch.as_tensor(np.arange(0, N, N // 16)[:16], device="cuda")
    fw = torch.zeros(N, 4, dtype=torch.float64, device="cuda")
    fw[torch.arange(nx - 1, N, nx, device="cuda"), 1] = wls[0].h
    fw = fw.reshape(-1)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in wls]
    ctxs, outs = [], []
    for wl, s in zip(wls, streams):
        with torch.cuda.stream(s):
            ctx = m.create(wl.dim, wl.ncell, wl.h)
            api.configure(ctx, wl, "fp64")
            m.set_checkpointing(ctx, True)
            m.set_timing(ctx, False)
            m.set_deferred_errors(ctx, True)
            p = torch.empty(N, dtype=torch.float64, device="cuda")
            fl = torch.empty(N * 4, dtype=torch.float64, device="cuda")
            dJdp = torch.zeros(N, dtype=torch.float64, device="cuda")
            grad = torch.empty(N, dtype=torch.float64, device="cuda")
        ctxs.append(ctx)
        outs.append((p, fl, dJdp, grad))
    torch.cuda.synchronize()
    t = 0.0
    for r in range(reps + 1):
        t0 = time.perf_counter()
        for ctx, wl, s, (p, fl, dJdp, grad) in zip(ctxs, wls, streams, outs):
            with torch.cuda.stream(s):
                m.build_basis(ctx)
                m.solve_interface(ctx)
                m.smooth(ctx, wl.nsmooth)
                m.get_solution(ctx, p, fl)
                dJdp[obs] = p[obs] - 0.1
                m.adjoint(ctx, dJdp, fw, grad)
        for ctx in ctxs:
            m.wait(ctx)
        torch.cuda.synchronize()
        if r:  # the first round builds the plans and allocates
            t += (time.perf_counter() - t0) / reps
    for ctx in ctxs:
        m.destroy(ctx)
    return {"members": members, "streams": members, "ms_per_batch": round(t * 1e3, 3),
            "ms_per_member": round(t * 1e3 / members, 4),
            "fine_cells_per_s_forward_and_gradient": members * N / t}


def boxes(wl):
    """Oversampled boxes (cells per axis), seeds per box, subdomain cells."""
    import numpy as np
    out = []
    M = [wl.ncell[a] // wl.sub[a] for a in range(wl.dim)]
    per_side = {"const": 1, "linear": wl.dim, "fine": None}[wl.space]
    for idx in np.ndindex(*M[::-1]):
        ic = idx[::-1]
        dims, nseed = [], 0
        for a in range(wl.dim):
            lo = max(ic[a] * wl.sub[a] - wl.overlap, 0)
            hi = min((ic[a] + 1) * wl.sub[a] + wl.overlap, wl.ncell[a])
            dims.append(hi - lo)
        for a in range(wl.dim):
            for s in (0, 1):
                t = ic[a] + (1 if s else -1)
                if 0 <= t < M[a]:
                    if per_side is None:
                        n = 1
                        for b in range(wl.dim):
                            if b != a:
                                n *= wl.sub[b]
                        nseed += n
                    else:
                        nseed += per_side
        out.append((dims, nseed))
    return out


def roofline(wl, form, phases, st):
    """Roofline of the dominant kernel of one solve (largest device time)."""
    import numpy as np
    bx = boxes(wl)
    word = 4 if form == "fp32_refine" else 8
    solves = max(st["refine_max_iters"], 1) if form == "fp32_refine" else 1
    n_launch = max(st["n_smooth_launches"], 1)
    phases_per_launch = max(st["n_smooth_phases"], 1) / n_launch
    t_smooth_launch = phases["ms_smooth"] / n_launch * 1e-3
    t_basis = phases["ms_basis_kernel"] * 1e-3
    cand = {"basis": t_basis, "smooth": phases["ms_smooth"] * 1e-3}
    dom = max(cand, key=cand.get)
    S = wl.sub
    if dom == "smooth":
        # algorithmic bytes of one colour phase, averaged over the colours:
        # cached block inverses (once per solve; FP64: symmetric, lower
        # triangles) + block couplings, K and p with a one-cell halo, f;
        # written: p on Omega_i and its Gamma fluxes
        total = 0.0
        for dims, _ in bx:
            nb, nblk = dims[0], int(np.prod(dims[1:]))
            ncb = nb * nblk
            halo = int(np.prod([d + 2 for d in dims]))
            blk = nb * nb if form == "fp32_refine" else nb * (nb + 1) // 2
            total += solves * nblk * blk * word + ncb * 8 + 2 * halo * 8 + ncb * 8
            total += int(np.prod(S)) * 8 + 2 * wl.dim * int(np.prod(S[1:])) * 8
        # every box is solved once per sweep of 2^d colour phases; a launch
        # runs one phase, or all phases of the call in the persistent form
        per_launch = total / (2 ** wl.dim) * phases_per_launch
        achieved = per_launch / t_smooth_launch
        kern = "k_smooth32" if form == "fp32_refine" else "k_smooth_w"
        if st["smooth_persistent"]:
            kern = "k_smooth_grid"
        return {"kernel": kern, "bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": achieved / PEAK_HBM, "traffic": traffic(kern, wl),
                "work_per_launch": "%.0f bytes" % per_launch,
                "avg_launch_us": t_smooth_launch * 1e6}
    return local_roofline(wl, form, phases, st)


def local_roofline(wl, form, phases, st):
    """Roofline of the local kernel (basis boxes and particular problems in
    one launch), against the FP64 (or FP32) peak: executed flops of the
    block-dense elimination, and the band-factor flops of the method."""
    import numpy as np
    bx = boxes(wl)
    solves = max(st["refine_max_iters"], 1) if form == "fp32_refine" else 1
    t_basis = phases["ms_basis_kernel"] * 1e-3
    S = wl.sub
    # executed: Gauss-Jordan inverse of every line block (nb^3 FMA; in FP64
    # the blocks below the meeting block are eliminated from one end and
    # those above it from the other, still one inverse per block) and the
    # forward + backward block products of every right-hand side (2 nb^2 FMA
    # per block).  Band (algorithmic): n b^2 flops per factor, 4 n b per
    # right-hand side solve, with n the cells of the box and b = nb its
    # half-bandwidth in line order.
    flops = 0.0
    band = 0.0
    for dims, nseed in bx:
        nb, nblk = dims[0], int(np.prod(dims[1:]))
        flops += 2.0 * nblk * nb ** 3 + solves * 4.0 * nblk * nb * nb * nseed
        n = nb * nblk
        band += n * nb * nb + solves * 4.0 * n * nb * nseed
    for _ in range(int(np.prod(wl.ncell)) // int(np.prod(S))):
        nb, nblk = S[0], int(np.prod(S[1:]))
        flops += 2.0 * nblk * nb ** 3 + solves * 4.0 * nblk * nb * nb
        n = nb * nblk
        band += n * nb * nb + solves * 4.0 * n * nb
    achieved = flops / t_basis
    peak = PEAK_FP32 if form == "fp32_refine" else PEAK_FP64
    kern = "k_local32" if form == "fp32_refine" else "k_local_w"
    return {"kernel": kern, "bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic(kern, wl),
            "work_per_launch": "%.0f flop" % flops, "avg_launch_us": t_basis * 1e6,
            "band_flop_per_launch": band, "frac_band_algorithmic": band / t_basis / peak}


def calibrate_copy():
    """A plain copy kernel of known size: 256 MiB read and 256 MiB written per
    launch, three launches (reference for the HBM byte counters)."""
    import torch
    n = 256 * 1024 * 1024 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this MRCM-OS path has no multi-GPU form "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    from inputs import make_workload
    wl = make_workload(args.workload, overlap=args.overlap)
    forms = {}
    for form in ("fp32_refine", "fp64"):
        steps = args.steps if args.precision in ("best", form) else max(3, args.steps // 2)
        dt, ph, st, p, fl = time_solves(wl, form, steps, args.warmup, args.tol,
                                        args.smoothing == "persistent")
        forms[form] = {"dt": dt, "phases": ph, "stats": st, "p": p, "fl": fl, "steps": steps}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import mrcm as oracle_mrcm
        times = []
        ref = None
        # repeat full solves for about 10 s of CPU work (at least 3)
        while len(times) < 3 or (sum(times) < 10.0 and len(times) < 30):
            t = time.perf_counter()
            ref = oracle_mrcm.solve(wl)
            times.append(time.perf_counter() - t)
        tcpu = float(np.median(times))
        cpu = {"value": wl.ncells / tcpu, "unit": "fine cells/s", "cores": 1, "kind": "oracle",
               "sample": "median of %d full oracle solves of the benchmark workload "
                         "(%.2f s each, one thread; host has %s logical CPUs)"
                         % (len(times), tcpu, os.cpu_count())}
        rp, rf = ref.pressure(), ref.flux().ravel()
        for f in forms.values():
            f["err"] = {"flux_rel_l2": float(np.linalg.norm(f["fl"] - rf) / np.linalg.norm(rf)),
                        "pressure_rel_l2": float(np.linalg.norm(f["p"] - rp) / np.linalg.norm(rp))}
    if args.precision == "best":
        ok = [k for k, f in forms.items() if "err" not in f or f["err"]["flux_rel_l2"] <= FLUX_TOL]
        head = min(ok or forms, key=lambda k: forms[k]["dt"])
    else:
        head = args.precision
    other = "fp64" if head == "fp32_refine" else "fp32_refine"
    H, O = forms[head], forms[other]
    st = H["stats"]

    def form_summary(f, form):
        d = {"value": wl.ncells / f["dt"], "ms_per_step": f["dt"] * 1e3,
             "ms_per_solve_synchronous": round(f["stats"]["ms_per_solve_synchronous"], 4),
             "ms_synchronous_median_min_max": f["stats"]["ms_synchronous_median_min_max"],
             "phases_ms": {k: round(v, 4) for k, v in f["phases"].items()},
             "interface_share": round(f["phases"]["ms_interface"] / (f["dt"] * 1e3), 3),
             "one_time_ms": {"smoothing_autotune": round(f["stats"]["ms_autotune"], 3)},
             "roofline_local": local_roofline(wl, form, f["phases"], f["stats"])}
        if form == "fp32_refine":
            d["refine"] = {"tol": args.tol, "max_fp32_solves": f["stats"]["refine_max_iters"],
                           "max_backward_error": f["stats"]["refine_max_resid"]}
        if "err" in f:
            d["err_vs_oracle"] = f["err"]
        return d

    adj = None if args.no_extra else time_adjoint(make_workload("c5"), max(3, args.steps // 4))
    if adj is not None:
        adj["batch"] = time_batch(32, 3)
    extra = {}
    if not args.no_extra and args.workload == "c2":
        for l in (0, 2, 4):
            if l == args.overlap:
                continue
            w2 = make_workload(args.workload, overlap=l)
            d3, ph3, _, _, _ = time_solves(w2, head, max(3, args.steps // 2), 2, args.tol,
                                           args.smoothing == "persistent")
            extra["overlap_%d" % l] = {"ms_per_step": round(d3 * 1e3, 4), "value": w2.ncells / d3,
                                       **{k: round(v, 4) for k, v in ph3.items()}}
    line = {
        "metric": "fine cells/s per MRCM-OS solve, FP32+refine vs FP64, at flux err <=1e-6",
        "value": wl.ncells / H["dt"],
        "unit": "fine cells/s",
        "n_gpus": 1,
        "steps": H["steps"],
        "warmup": args.warmup,
        "ms_per_step": H["dt"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "fp32_refine" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %dx%d cells, subdomains %s, overlap %d, %s spaces, %d smoothing steps"
                   % (args.workload, wl.ncell[0], wl.ncell[1], "x".join(map(str, wl.sub)),
                      wl.overlap, wl.space, wl.nsmooth),
                   "smoothing": "one cooperative launch per call" if st["smooth_persistent"]
                   else "graph of per-colour launches",
                   "solves": "back to back, device errors read once per timed loop; "
                             "ms_per_solve_synchronous: each solve waits for its own",
                   "precision": head, "interface_unknowns": st["n_unknowns"],
                   "interface_solver": {1: "band_lu", 2: "block_cyclic_reduction"}[st["interface_solver"]]},
        head: form_summary(H, head),
        other: form_summary(O, other),
        "other_overlaps": extra,
        "adjoint": adj,
        "roofline": roofline(wl, head, H["phases"], st),
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()
