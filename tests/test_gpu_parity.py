"""GPU FP64 path vs the CPU oracle, element by element (relative L2 <= 1e-10
in pressure and flux, the bar for the FP64 form)."""
import sys

import numpy as np
import pytest

from inputs import make_workload

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SOLVER_NAME = {1: "band_lu", 2: "bcr"}


def _check(wl, nsmooth=None, tol=TOL, solver="auto"):
    from gpu_util import gpu_solve, oracle_solve, rel
    print("case", wl.name, wl.ncell, wl.sub, "l=%d" % wl.overlap, wl.space, "ns", nsmooth,
          "solver", solver, flush=True)
    p, fl, X, st = gpu_solve(wl, nsmooth=nsmooth, solver=solver)
    rp, rf, rX, _ = oracle_solve(wl, nsmooth=nsmooth)
    ep, ef = rel(p, rp), rel(fl, rf)
    used = SOLVER_NAME[st["interface_solver"]]
    print("  rel L2 p %.3e flux %.3e  (nX %d kl %d ku %d, interface solver %s)"
          % (ep, ef, st["n_unknowns"], st["band_kl"], st["band_ku"], used), flush=True)
    if solver != "auto":
        assert used == solver
    assert ep <= tol and ef <= tol
    return p, fl, X, rX


def _small(**kw):
    return make_workload("c1", scale=2).with_(beta_mode="alpha", beta_mbf=1.0, beta_smooth=1.0,
                                               sub=(8, 8)).with_(**kw)


@pytest.mark.parametrize("overlap", [0, 1, 2, 3])
@pytest.mark.parametrize("space", ["const", "linear"])
def test_small_mrcm_o(space, overlap):
    _, _, X, rX = _check(_small(space=space, overlap=overlap), nsmooth=0)
    assert np.linalg.norm(X - rX) <= 1e-9 * np.linalg.norm(rX)


@pytest.mark.parametrize("overlap", [0, 2, 3])
def test_small_with_smoothing(overlap):
    _check(_small(space="linear", overlap=overlap), nsmooth=3)


@pytest.mark.parametrize("suby,overlap", [(1, 0), (2, 0), (2, 1), (4, 3)])
def test_short_boxes_with_smoothing(suby, overlap):
    # boxes of 1 to 10 lines (truncated ones at the domain edge): the halves
    # of the two-ended box sweep are empty, one block or a few blocks long
    _check(_small(space="const", overlap=overlap, sub=(8, suby)), nsmooth=2)


@pytest.mark.parametrize("overlap", [0, 1, 2])
def test_fine_spaces_prop2(overlap):
    _check(_small(space="fine", overlap=overlap), nsmooth=0)


def test_c1_full():
    _check(make_workload("c1"))


@pytest.mark.parametrize("overlap", [0, 2, 4])
def test_c2_scaled_pure_neumann(overlap):
    _check(make_workload("c2", scale=4, overlap=overlap))


@pytest.mark.parametrize("overlap", [0, 2, 4])
def test_c2_full(overlap):
    _check(make_workload("c2", overlap=overlap))


# The two interface solvers on the same systems (the natural-order banded LU
# and the block cyclic reduction over subdomain layers).
@pytest.mark.parametrize("solver", ["band_lu", "bcr"])
@pytest.mark.parametrize("case", ["small_linear_l2", "small_const_l0", "c1", "c2_scaled_l2",
                                  "c2_full_l0", "c2_full_l4", "c5", "c3_scaled"])
def test_interface_solvers(case, solver):
    wl = {
        "small_linear_l2": lambda: _small(space="linear", overlap=2),
        "small_const_l0": lambda: _small(space="const", overlap=0),
        "c1": lambda: make_workload("c1"),
        "c2_scaled_l2": lambda: make_workload("c2", scale=4, overlap=2),
        "c2_full_l0": lambda: make_workload("c2", overlap=0),
        "c2_full_l4": lambda: make_workload("c2", overlap=4),
        "c5": lambda: make_workload("c5"),
        "c3_scaled": lambda: make_workload("c3", scale=4),
    }[case]()
    ns = 0 if case.startswith("small") else None
    _, _, X, rX = _check(wl, nsmooth=ns, solver=solver)
    assert np.linalg.norm(X - rX) <= 1e-9 * np.linalg.norm(rX)


# Layer blocks above 128 unknowns (32 subdomains of 8 x 8 per layer, linear
# spaces: 248 unknowns) use the two-by-two block inverse.
@pytest.mark.parametrize("overlap", [0, 2])
def test_bcr_large_layer_blocks(overlap):
    wl = make_workload("c2", overlap=overlap).with_(sub=(8, 8))
    _, _, X, rX = _check(wl, nsmooth=2, solver="bcr")
    assert np.linalg.norm(X - rX) <= 1e-9 * np.linalg.norm(rX)


# Full-size channel workload: 1024 x 1024 cells, 64 x 64 subdomains,
# 16128 interface unknowns in 64 layers of up to 256 (about a minute of
# oracle time).
def test_c3_full():
    _check(make_workload("c3"))


def test_three_dimensional_small():
    _check(make_workload("c4", scale=8), nsmooth=1)


# ------------------------------------------------------------ FP32 + refinement
def _check32(wl, nsmooth=None, tol_flux=1e-6, tol_p=1e-6):
    from gpu_util import gpu_solve, oracle_solve, rel
    print("case fp32", wl.name, wl.ncell, "l=%d" % wl.overlap, wl.space, flush=True)
    p, fl, X, st = gpu_solve(wl, precision="fp32_refine", nsmooth=nsmooth, tol=1e-12, max_refine=30)
    rp, rf, _, _ = oracle_solve(wl, nsmooth=nsmooth)
    ep, ef = rel(p, rp), rel(fl, rf)
    print("  fp32+refine rel L2 p %.3e flux %.3e  refine iters %d backward err %.2e"
          % (ep, ef, st["refine_max_iters"], st["refine_max_resid"]), flush=True)
    assert ef <= tol_flux and ep <= tol_p
    assert st["refine_max_resid"] <= 1e-12
    return ep, ef


@pytest.mark.parametrize("overlap", [0, 2])
def test_fp32_refine_small(overlap):
    _check32(_small(space="linear", overlap=overlap), nsmooth=2)


def test_fp32_refine_c1():
    _check32(make_workload("c1"))


@pytest.mark.parametrize("overlap", [0, 2, 4])
def test_fp32_refine_c2_full(overlap):
    _check32(make_workload("c2", overlap=overlap))


def test_fp32_refine_c3_full():
    """The channel workload at full size (1024 x 1024, contrast 1e4) in the
    FP32 + refinement form, against the oracle: flux within 1e-6."""
    _check32(make_workload("c3"))


# ------------------------------------------------- smoothing execution forms
def _smooth_trace(wl, use_graph, threads, steps, precision="fp64", persistent=None):
    """Pressure and flux after each mrcm_smooth call (eager reads between
    the calls, so graph replays alternate with other device work).
    persistent: None, or (on, max_groups) for the one-launch form."""
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    out = []
    try:
        api.configure(ctx, wl, precision, tol=1e-12, max_refine=30)
        m.set_smoothing(ctx, use_graph, threads)
        if persistent is not None:
            m.set_smoothing_persistent(ctx, *persistent)
        m.build_basis(ctx)
        m.solve_interface(ctx)
        for n in steps:
            m.smooth(ctx, n)
            out.append((m.get_pressure(ctx).cpu().numpy(), m.get_flux(ctx).cpu().numpy()))
        st = m.get_stats(ctx)
        torch.cuda.synchronize()
    finally:
        m.destroy(ctx)
    return out, st


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_smoothing_graph_and_thread_variants_agree_exactly(precision):
    """Every threads-per-box variant and every graph replay gives results
    bit-identical to plain launches after the same number of steps."""
    wl = make_workload("c2", scale=4, overlap=2)
    steps = [2, 1, 2, 1]
    ref, _ = _smooth_trace(wl, False, 64, steps, precision)
    for use_graph, threads in [(False, 128), (False, 256), (True, 0), (True, 64)]:
        got, st = _smooth_trace(wl, use_graph, threads, steps, precision)
        print("graph", use_graph, "threads", threads, "->", st["smooth_threads"],
              "autotune ms %.3f" % st["ms_autotune"], flush=True)
        assert st["smooth_graph"] == int(use_graph)
        assert st["smooth_threads"] in (64, 128, 256)
        for (p, fl), (rp, rf) in zip(got, ref):
            assert np.array_equal(p, rp) and np.array_equal(fl, rf)


@pytest.mark.parametrize("overlap", [2, 0])
def test_persistent_smoothing_agrees_exactly(overlap):
    """All colour phases of a call in one cooperative launch (Steps 6-7 with
    a device-wide barrier between colours) give results bit-identical to
    one launch per phase, also when the grid is capped so that every
    workgroup loops over several boxes of a colour, and for every
    threads-per-box variant."""
    wl = make_workload("c2", scale=4, overlap=overlap)
    steps = [2, 1, 3]
    ref, _ = _smooth_trace(wl, False, 256, steps)
    for threads, groups in [(256, 0), (128, 0), (64, 0), (256, 3), (128, 1)]:
        got, st = _smooth_trace(wl, False, threads, steps, persistent=(True, groups))
        print("persistent threads", threads, "max_groups", groups, "used", st["smooth_persistent"],
              "launches", st["n_smooth_launches"], "phases", st["n_smooth_phases"], flush=True)
        assert st["smooth_persistent"] == 1 and st["n_smooth_launches"] == 1
        assert st["n_smooth_phases"] == steps[-1] * 2 ** wl.dim
        for (p, fl), (rp, rf) in zip(got, ref):
            assert np.array_equal(p, rp) and np.array_equal(fl, rf)


def test_get_solution_matches_separate_outputs():
    """mrcm_get_solution gives the pressure and flux of mrcm_get_pressure and
    mrcm_get_flux, bit for bit, and smoothing calls with changing step
    counts (each a graph of its own, here without phase-timing events) agree
    with one call of their sum."""
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    wl = make_workload("c2", scale=4, overlap=2)
    out = []
    for steps in ([3], [1, 2]):
        ctx = m.create(wl.dim, wl.ncell, wl.h)
        try:
            api.configure(ctx, wl, "fp64")
            m.set_timing(ctx, len(steps) == 1)
            m.build_basis(ctx)
            m.solve_interface(ctx)
            for n in steps:
                m.smooth(ctx, n)
            p, fl = m.get_solution(ctx)
            p2 = m.get_pressure(ctx)
            fl2 = m.get_flux(ctx)
            out.append((p.cpu().numpy(), fl.cpu().numpy()))
            assert np.array_equal(out[-1][0], p2.cpu().numpy())
            assert np.array_equal(out[-1][1], fl2.cpu().numpy())
        finally:
            m.destroy(ctx)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
