"""3-D workloads in the FP32 + refinement form against the FP64 CPU oracle:
FP32 plane inverses of the diagonally scaled box matrices, every local
solve refined in FP64 to a componentwise backward error of 1e-12; the
relative L2 error of flux and pressure within 1e-6 (the precision form's
bound).  Covers the layered Gaussian-field recipe at reduced and at full
size, linear interface spaces, a smoothing Robin parameter that differs
from the basis one (Step 6), a diagonal permeability tensor, boxes of more
planes than the kernels hold in registers, plane sizes for one, two and
four waves per box (aligned and unaligned rows), no oversampling, and the
no-convergence report."""
import os

import numpy as np
import pytest

from inputs import make_workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL32 = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check32(wl, nsmooth=None, tol=TOL32):
    from gpu_util import gpu_solve, oracle_solve, rel
    print("case fp32", wl.name, wl.ncell, wl.sub, "l=%d" % wl.overlap, wl.space,
          "alpha %g/%g" % (wl.beta_mbf, wl.beta_smooth), flush=True)
    p, fl, X, st = gpu_solve(wl, precision="fp32_refine", nsmooth=nsmooth, tol=1e-12, max_refine=30)
    rp, rf, rX, _ = oracle_solve(wl, nsmooth=nsmooth)
    ep, ef, ex = rel(p, rp), rel(fl, rf), rel(X, rX)
    print("  fp32+refine rel L2 p %.3e flux %.3e X %.3e; FP32 solves <= %d, backward error %.2e"
          % (ep, ef, ex, st["refine_max_iters"], st["refine_max_resid"]), flush=True)
    assert st["refine_max_resid"] <= 1e-12
    assert 2 <= st["refine_max_iters"] <= 31
    assert ep <= tol and ef <= tol
    return ep, ef


@pytest.mark.parametrize("scale", [4, 2])
def test_fp32_refine_3d_recipe(scale):
    # scale 4: 16 x 56 x 20 cells, 280 subdomains; scale 2: 32 x 112 x 40
    # cells, 2240 subdomains (the two-level interface solver)
    _check32(make_workload("c4", scale=scale))


def test_fp32_refine_3d_linear_spaces():
    _check32(make_workload("c4", scale=8, space="linear"), nsmooth=1)


def test_fp32_refine_3d_distinct_smoothing_parameter():
    # Step 6: the oversampled boxes factored once more (FP32) with alpha = 1
    wl = make_workload("c4", scale=8).with_(beta_mode="alpha", beta_mbf=1e-2, beta_smooth=1.0, nsmooth=2)
    _check32(wl)


def test_fp32_refine_3d_tensor():
    rng = np.random.default_rng(7)
    wl = make_workload("c4", scale=8)
    wl = wl.with_tensor([0.0] + [rng.normal(size=wl.logk.shape) for _ in range(2)])
    _check32(wl, nsmooth=1)


def test_fp32_refine_3d_boxes_beyond_the_register_cache():
    # subdomains of 4 x 4 x 5 cells with overlap 2: boxes of up to 9 planes
    # of 64 cells, so the ninth plane's inverse is read back from memory
    wl = make_workload("c4", scale=4).with_(sub=(4, 4, 5))
    _check32(wl, nsmooth=2)


def test_fp32_refine_3d_agrees_with_fp64():
    from gpu_util import gpu_solve, rel
    wl = make_workload("c4", scale=4)
    p64, f64, _, _ = gpu_solve(wl, precision="fp64")
    p32, f32, _, st = gpu_solve(wl, precision="fp32_refine", tol=1e-12, max_refine=30)
    print("  fp32+refine against fp64 on the device: p %.2e flux %.2e" % (rel(p32, p64), rel(f32, f64)),
          flush=True)
    assert rel(f32, f64) <= TOL32 and rel(p32, p64) <= TOL32


def test_fp32_refine_c4_full_against_oracle_samples():
    """Full size: 64 x 224 x 80 cells, 17,920 subdomains, 102,848 interface
    unknowns, 3 smoothing steps, FP32 + refinement; the oracle's solution at
    4096 seeded cells against the device's."""
    from gpu_util import gpu_solve
    ref = np.load(os.path.join(GOLDEN, "c4_full_samples.npz"))
    wl = make_workload("c4")
    p, fl, X, st = gpu_solve(wl, precision="fp32_refine", tol=1e-12, max_refine=30)
    cells = ref["cells"]
    fl = fl.reshape(wl.ncells, 6)
    ep = np.linalg.norm(p[cells] - ref["pressure"]) / np.linalg.norm(ref["pressure"])
    ef = np.linalg.norm(fl[cells] - ref["flux"]) / np.linalg.norm(ref["flux"])
    print("  full c4 fp32+refine: sampled rel L2 p %.3e flux %.3e; FP32 solves <= %d, backward "
          "error %.2e" % (ep, ef, st["refine_max_iters"], st["refine_max_resid"]), flush=True)
    assert st["refine_max_resid"] <= 1e-12
    assert ep <= TOL32 and ef <= TOL32


def test_fp32_refine_3d_reports_no_convergence():
    """One FP32 solve allowed (max_refine 0) against a backward-error bound
    no FP32 solve meets: the solve reports MRCM_ENOCONV."""
    from gpu_util import gpu_solve
    wl = make_workload("c4", scale=8)
    with pytest.raises(RuntimeError, match="MRCM_ENOCONV"):
        gpu_solve(wl, precision="fp32_refine", tol=1e-15, max_refine=0)


@pytest.mark.parametrize("sub,overlap", [((4, 7, 4), 1), ((4, 7, 4), 0), ((4, 4, 4), 0), ((2, 7, 8), 1)])
def test_fp32_refine_3d_box_shapes(sub, overlap):
    # planes of 54, 45, 40 cells (rows of the stored inverses not 16-byte
    # aligned), of 28 (two waves per box) and 16 (one wave), no oversampling
    # (smoothing data from the neighbours' Gamma fluxes), and boxes whose
    # oversampling is truncated on both sides of an axis
    wl = make_workload("c4", scale=8).with_(sub=sub, overlap=overlap, nsmooth=2)
    _check32(wl)
