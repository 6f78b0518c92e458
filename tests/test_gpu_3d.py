"""3-D workloads on the device against the CPU oracle: the two-level
interface solver (outer layers of subdomains along the axis with the most
subdomains, one batched block cyclic reduction of all layers' own systems,
then the reduced system over the gaps between layers) on the layered
Gaussian-field recipe at reduced and at full size, and piecewise-linear
interface spaces in 3-D (three seeds per side)."""
import os

import numpy as np
import pytest

from inputs import make_workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(wl, solver="auto", nsmooth=None, expect=None):
    from gpu_util import gpu_solve, oracle_solve, rel
    print("case", wl.name, wl.ncell, wl.sub, "l=%d" % wl.overlap, wl.space, "solver", solver,
          flush=True)
    p, fl, X, st = gpu_solve(wl, nsmooth=nsmooth, solver=solver)
    rp, rf, rX, _ = oracle_solve(wl, nsmooth=nsmooth)
    ep, ef, ex = rel(p, rp), rel(fl, rf), rel(X, rX)
    print("  rel L2 p %.3e flux %.3e X %.3e (nX %d, interface solver %d, backward error %.1e)"
          % (ep, ef, ex, st["n_unknowns"], st["interface_solver"], st["interface_residual"]),
          flush=True)
    if expect is not None:
        assert st["interface_solver"] == expect
    assert ex <= 1e-9
    assert ep <= TOL and ef <= TOL
    return X


@pytest.mark.parametrize("scale", [4, 2])
def test_layered_solver_on_the_3d_recipe(scale):
    # scale 4: 16 x 56 x 20 cells, 280 subdomains; scale 2: 32 x 112 x 40
    # cells, 2240 subdomains, 12272 unknowns (layers of the cyclic reduction
    # would exceed 256 unknowns: the automatic choice is the two-level solver)
    _check(make_workload("c4", scale=scale), solver="auto", expect=3)


def test_layered_equals_the_cyclic_reduction_where_both_apply():
    wl = make_workload("c4", scale=8)
    x_bcr = _check(wl, solver="bcr", nsmooth=1, expect=2)
    x_lay = _check(wl, solver="layered", nsmooth=1, expect=3)
    assert np.linalg.norm(x_lay - x_bcr) <= 1e-12 * np.linalg.norm(x_bcr)


@pytest.mark.parametrize("scale,solver", [(8, "auto"), (4, "layered")])
def test_three_dimensional_linear_spaces(scale, solver):
    _check(make_workload("c4", scale=scale, space="linear"), solver=solver, nsmooth=1)


def test_c4_full_against_oracle_samples():
    """Full size: 64 x 224 x 80 cells, 17,920 subdomains, 102,848 interface
    unknowns, 3 smoothing steps.  The oracle's solution at 4096 seeded cells
    (tests/golden/make_c4_samples.py) against the device's."""
    from gpu_util import gpu_solve
    ref = np.load(os.path.join(GOLDEN, "c4_full_samples.npz"))
    wl = make_workload("c4")
    p, fl, X, st = gpu_solve(wl)
    assert st["n_unknowns"] == int(ref["n_unknowns"]) and st["interface_solver"] == 3
    cells = ref["cells"]
    fl = fl.reshape(wl.ncells, 6)
    dp = p[cells] - ref["pressure"]
    df = fl[cells] - ref["flux"]
    ep = np.linalg.norm(dp) / np.linalg.norm(ref["pressure"])
    ef = np.linalg.norm(df) / np.linalg.norm(ref["flux"])
    print("  full c4: sampled rel L2 p %.3e flux %.3e; max |dp| %.2e of ||p||_2/sqrt(N) %.2e; "
          "backward error %.1e" % (ep, ef, np.abs(dp).max(),
                                   float(ref["pressure_norm"]) / np.sqrt(wl.ncells),
                                   st["interface_residual"]), flush=True)
    assert ep <= TOL and ef <= TOL
    # the whole fields' norms agree as well
    assert abs(np.linalg.norm(p) - float(ref["pressure_norm"])) <= TOL * float(ref["pressure_norm"])
    assert abs(np.linalg.norm(fl) - float(ref["flux_norm"])) <= TOL * float(ref["flux_norm"])
