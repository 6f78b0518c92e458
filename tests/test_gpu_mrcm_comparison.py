"""The original MRCM (MRCM-O with no oversampling, linear spaces, no
smoothing: two multipliers per interface) beside MRCM-OS on the device, on
the log-normal recipe: every configuration against the oracle's solution of
the same configuration, and the errors against the fine-grid solution.  At
64 x 64 cells (4 x 4 subdomains) they fall in the order the paper reports
(Section 5: MRCM-OS with oversampling 4h and four smoothing steps more than
an order of magnitude below MRCM in flux); at full size (256 x 256 cells,
the paper's 16 x 16 decomposition) the errors are recorded, and MRCM-OS
does not beat MRCM there (the design notes give the figures)."""
import pytest

from inputs import make_workload

pytestmark = pytest.mark.gpu

CONFIGS = {
    "MRCM": dict(overlap=0, space="linear", nsmooth=0),
    "OC-2,2S": dict(overlap=2, space="const", nsmooth=2),
    "OL-2,2S": dict(overlap=2, space="linear", nsmooth=2),
    "OL-4,4S": dict(overlap=4, space="linear", nsmooth=4),
}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _compare(base):
    from gpu_util import gpu_solve, oracle_solve, rel
    from oracle import mrcm
    fp, ff = mrcm.fine(base)
    err = {}
    for name, cfg in CONFIGS.items():
        wl = base.with_(**cfg)
        print("case", name, wl.ncell, wl.sub, "l=%d" % wl.overlap, wl.space, "N_s=%d" % wl.nsmooth,
              flush=True)
        p, fl, _, st = gpu_solve(wl)
        rp, rf, _, _ = oracle_solve(wl)
        assert rel(p, rp) <= 1e-10 and rel(fl, rf) <= 1e-10
        err[name] = (rel(p, fp), rel(fl, ff))
        print("  %s: %d interface unknowns; against the fine solution p %.3e flux %.3e"
              % (name, st["n_unknowns"], err[name][0], err[name][1]), flush=True)
    return err


def test_mrcm_and_mrcm_os_small():
    err = _compare(make_workload("c5", scale=4))
    assert err["OL-4,4S"][1] * 10.0 <= err["MRCM"][1]
    assert err["OC-2,2S"][1] < err["MRCM"][1]


def test_mrcm_and_mrcm_os_full_size():
    _compare(make_workload("c5"))
