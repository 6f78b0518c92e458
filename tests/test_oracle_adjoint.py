"""Pins of the differentiable oracle (oracle/mrcm_torch.py), the CPU FP64
adjoint of the MRCM-OS map log K -> (pressure, face velocities):

* its forward pass equals the numpy oracle (independent arithmetic for
  every K-dependent quantity) on small cases of every kind of boundary,
  overlap and interface space;
* its reverse-mode gradient equals central finite differences along random
  directions (step 1e-5 in log K)."""
import numpy as np
import pytest
import torch

from inputs import make_workload
from oracle import mrcm
from oracle import mrcm_torch as MT


def _small(**kw):
    return make_workload("c1", scale=2).with_(beta_mode="alpha", beta_mbf=1.0, beta_smooth=1.0,
                                               sub=(8, 8)).with_(**kw)


CASES = {
    "const_l2_dirichlet": lambda: _small(space="const", overlap=2),
    "linear_l0": lambda: _small(space="linear", overlap=0),
    "linear_l3": lambda: _small(space="linear", overlap=3),
    "neumann_wells_l2": lambda: make_workload("c2", scale=8, overlap=2),
    "neumann_wells_l0": lambda: make_workload("c2", scale=8, overlap=0),
    "beta_const": lambda: make_workload("c1", scale=2),
    # Algorithm 1, Step 6: smoothing boxes factored with their own parameter
    "alpha_distinct_small_l2": lambda: _small(space="const", overlap=2, beta_mbf=1e-2),
    "alpha_distinct_large_l0": lambda: _small(space="linear", overlap=0, beta_mbf=1e2),
    "alpha_distinct_wells_l3": lambda: make_workload("c2", scale=8, overlap=3).with_(beta_mbf=1e2),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_forward_matches_numpy_oracle(case):
    wl = CASES[case]()
    ref = mrcm.solve(wl, nsmooth=2)
    tm = MT.solve(wl, nsmooth=2)
    p, f = tm.pressure().numpy(), tm.flux().numpy().ravel()
    rp, rf = ref.pressure(), ref.flux().ravel()
    assert np.linalg.norm(p - rp) <= 1e-11 * np.linalg.norm(rp)
    assert np.linalg.norm(f - rf) <= 1e-11 * np.linalg.norm(rf)


def _objective(wl, nsmooth):
    def J(lk):
        m = MT.TorchMRCM(wl, lk).run(nsmooth)
        p, fl = m.pressure(), m.flux()
        obs = torch.arange(0, m.N, 97)
        return 0.5 * ((p[obs] - 0.1) ** 2).sum() + MT.outflow(fl, m, 1)
    return J


@pytest.mark.parametrize("case", ["const_l2_dirichlet", "linear_l0", "neumann_wells_l2", "beta_const"])
def test_gradient_matches_finite_differences(case):
    wl = CASES[case]()
    J = _objective(wl, 2)
    lk0 = torch.tensor(wl.logk.ravel(), dtype=torch.float64)
    lk = lk0.clone().requires_grad_(True)
    J(lk).backward()
    g = lk.grad.numpy()
    rng = np.random.default_rng(7)
    eps = 1e-5
    for _ in range(2):
        v = rng.standard_normal(lk0.numel())
        with torch.no_grad():
            fd = (J(lk0 + eps * torch.tensor(v)).item() - J(lk0 - eps * torch.tensor(v)).item()) / (2 * eps)
        assert abs(g @ v - fd) <= 1e-6 * abs(fd)
