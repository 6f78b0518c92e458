"""Algorithm 1, Step 6 and Section 5's study of the Robin parameter: basis
functions with alpha_mbf from 1e-8 to 1e8, smoothing with alpha_sm = 1 (the
oversampled boxes factored a second time with the smoothing parameter),
against the CPU oracle element by element.

FP64 bar: relative L2 <= 1e-10 in pressure and flux where the interface
system is well conditioned.  Large alpha_mbf makes the interface system
ill-conditioned (condition numbers 1e5 at 1e4, 1e9 to 3e10 at 1e8, measured
on the oracle's own matrix): a direct FP64 solve then carries a forward
error of order cond(G) times the unit roundoff, so the bar becomes
max(1e-10, 1e-14 cond(G)), a backward error of 1e-14 (about 50 ulps)
propagated through the system.  Above alpha_mbf = 1e4 the library's
automatic choice is the pivoted banded LU: the cyclic reduction, which does
not pivot, breaks down there, and its check reports it."""
import numpy as np
import pytest

from inputs import make_workload

pytestmark = pytest.mark.gpu

ALPHAS = [1e-8, 1e-4, 1e-2, 1.0, 1e2, 1e4, 1e8]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _wl(kind, alpha):
    if kind == "const_l2":
        wl = make_workload("c5", scale=2)                       # 128 x 128, 8 x 8 subdomains
    else:
        wl = make_workload("c2", scale=4, overlap=2)            # 64 x 64, wells, linear spaces
    return wl.with_(beta_mode="alpha", beta_mbf=alpha, beta_smooth=1.0, nsmooth=3)


def _oracle_sensitivity(wl):
    """How far the oracle's own answer moves with the rounding of its
    interface solve: the same system solved by a dense LU (LAPACK) instead
    of the sparse one, then combined and smoothed alike."""
    from oracle import mrcm
    from gpu_util import oracle_solve, rel
    rp, rf, _, _ = oracle_solve(wl)
    s = mrcm.MRCM(wl)
    s.build_basis()
    s.particular()
    s.assemble_interface()
    s.X = np.linalg.solve(s.G.toarray(), s.r)
    s.combine()
    s.smooth(wl.nsmooth)
    return rel(s.pressure(), rp), rel(s.flux().ravel(), rf)


def _interface_condition(wl):
    """2-norm condition number of the oracle's interface matrix."""
    from oracle import mrcm
    s = mrcm.MRCM(wl)
    s.build_basis()
    s.particular()
    G, _ = s.assemble_interface()
    return float(np.linalg.cond(G.toarray()))


def _run(wl, precision="fp64", solver="auto", check=None):
    from gpu_util import gpu_solve, oracle_solve, rel
    print("case", wl.name, wl.ncell, "l=%d" % wl.overlap, wl.space, "alpha_mbf %.0e" % wl.beta_mbf,
          "alpha_sm %.0e" % wl.beta_smooth, precision, solver, flush=True)
    p, fl, X, st = gpu_solve(wl, precision=precision, tol=1e-12, max_refine=30, solver=solver,
                             check=check)
    rp, rf, rX, _ = oracle_solve(wl)
    ep, ef = rel(p, rp), rel(fl, rf)
    print("  rel L2 p %.3e flux %.3e X %.3e; interface backward error %.2e"
          % (ep, ef, rel(X, rX), st["interface_residual"]), flush=True)
    if check is None:
        assert st["interface_residual"] <= 1e-5
    return ep, ef, st


# The library's automatic interface solver: the cyclic reduction up to
# alpha_mbf = 1e4, the pivoted banded LU above (the reduction's breakdown
# there is detected, see the test below).
@pytest.mark.parametrize("alpha", ALPHAS)
@pytest.mark.parametrize("kind", ["const_l2", "linear_l2_wells"])
def test_alpha_sweep_fp64(kind, alpha):
    wl = _wl(kind, alpha)
    ep, ef, st = _run(wl)
    assert st["interface_solver"] == (1 if alpha > 1e4 else 2)
    cond = _interface_condition(wl)
    sp, sf = _oracle_sensitivity(wl)
    bar = max(1e-10, 1e-14 * cond)
    print("  cond(G) %.2e  bar %.1e  oracle sensitivity p %.3e flux %.3e" % (cond, bar, sp, sf),
          flush=True)
    assert ep <= bar and ef <= bar
    if alpha <= 1e2:
        assert ep <= 1e-10 and ef <= 1e-10


@pytest.mark.parametrize("alpha", [1e-4, 1e4])
def test_alpha_sweep_fp32_refine(alpha):
    ep, ef, _ = _run(_wl("const_l2", alpha), "fp32_refine")
    assert ef <= 1e-6 and ep <= 1e-6


@pytest.mark.parametrize("kind", ["const_l2", "linear_l2_wells"])
def test_interface_check_flags_an_inaccurate_reduction(kind):
    """alpha_mbf = 1e8 through the cyclic reduction with the check off: the
    measured backward error decides; with the check on, a solve whose
    backward error exceeds the default tolerance (1e-5) is reported as
    MRCM_ESINGULAR and one below it passes."""
    import paper_2404_13811_amd as m
    wl = _wl(kind, 1e8)
    _, _, st = _run(wl, solver="bcr", check=0.0)
    be = st["interface_residual"]
    print("  cyclic reduction at alpha_mbf 1e8: backward error %.2e" % be, flush=True)
    if be > 1e-5:
        with pytest.raises(m.MRCMError) as err:
            m.solve_workload(wl, solver="bcr")
        assert err.value.status == 8  # MRCM_ESINGULAR
    else:
        m.solve_workload(wl, solver="bcr")
