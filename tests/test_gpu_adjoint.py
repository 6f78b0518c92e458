"""Device adjoint (mrcm_adjoint) against the CPU FP64 adjoint of the
differentiable oracle (relative L2 <= 1e-8) and against central finite
differences of the device forward map (relative 1e-4); the FP32+refine form
(FP32 local factors, every local solve refined in FP64 to a componentwise
backward error of 1e-12) against the same oracle gradient."""
import numpy as np
import pytest

from inputs import make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _small(**kw):
    return make_workload("c1", scale=2).with_(beta_mode="alpha", beta_mbf=1.0, beta_smooth=1.0,
                                               sub=(8, 8)).with_(**kw)


def _weights(wl, n_obs=16):
    """J = 1/2 sum_obs (p_o - d_o)^2 + sum over the +x boundary faces of |e| u.n"""
    nx, ny = wl.ncell
    N = nx * ny
    obs = np.arange(0, N, max(1, N // n_obs))[:n_obs]
    d = np.full(obs.size, 0.1)
    fw = np.zeros((N, 4))
    cells = np.arange(N)
    fw[cells[cells % nx == nx - 1], 1] = wl.h  # |e| in 2-D
    return obs, d, fw


def _gpu_grad(wl, nsmooth, precision="fp64"):
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    obs, d, fw = _weights(wl)
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    try:
        api.configure(ctx, wl, precision)
        m.set_checkpointing(ctx, True)
        m.build_basis(ctx)
        m.solve_interface(ctx)
        m.smooth(ctx, nsmooth)
        p = m.get_pressure(ctx)
        fl = m.get_flux(ctx)
        dJdp = torch.zeros_like(p)
        dJdp[torch.as_tensor(obs, device="cuda")] = p[torch.as_tensor(obs, device="cuda")] - torch.as_tensor(d, device="cuda")
        dJdf = torch.as_tensor(fw.ravel(), device="cuda")
        g = m.adjoint(ctx, dJdp, dJdf).cpu().numpy()
        pn, fn = p.cpu().numpy(), fl.cpu().numpy()
        J = 0.5 * np.sum((pn[obs] - d) ** 2) + np.dot(fw.ravel(), fn)
    finally:
        m.destroy(ctx)
    return J, g


def _oracle_grad(wl, nsmooth):
    import torch
    from oracle import mrcm_torch as MT
    obs, d, fw = _weights(wl)
    lk = torch.tensor(wl.logk.ravel(), dtype=torch.float64, requires_grad=True)
    mm = MT.TorchMRCM(wl, lk).run(nsmooth)
    p, fl = mm.pressure(), mm.flux()
    J = 0.5 * ((p[torch.as_tensor(obs)] - torch.as_tensor(d)) ** 2).sum() + (torch.as_tensor(fw) * fl).sum()
    J.backward()
    return J.item(), lk.grad.numpy()


CASES = {
    "const_l2_dirichlet": (lambda: _small(space="const", overlap=2), 2),
    "linear_l0": (lambda: _small(space="linear", overlap=0), 2),
    "linear_l3": (lambda: _small(space="linear", overlap=3), 3),
    "neumann_wells_l2": (lambda: make_workload("c2", scale=8, overlap=2), 2),
    "neumann_wells_l0": (lambda: make_workload("c2", scale=8, overlap=0), 2),
    "beta_const": (lambda: make_workload("c1", scale=2), 2),
    "no_smoothing": (lambda: _small(space="linear", overlap=2), 0),
    # subdomains one and two cells thick: both sides of an axis touch the
    # same cells in the box right-hand sides and their adjoints
    "thin_rows_l0": (lambda: _small(space="const", overlap=0, sub=(8, 1)), 2),
    "thin_rows_l1": (lambda: _small(space="const", overlap=1, sub=(8, 2)), 2),
    # 64 x 64 cells, 4 x 4 subdomains of 16 x 16 (the first recipe at full
    # size, alpha = 1)
    "grid64_sub4x4": (lambda: make_workload("c1").with_(beta_mode="alpha", beta_mbf=1.0,
                                                         beta_smooth=1.0), 2),
    # one full member of the batch workload: 256 x 256 cells, 16 x 16
    # subdomains, overlap 2, five smoothing steps (about 30 s on the CPU)
    "batch_member_256": (lambda: make_workload("c5"), 5),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_adjoint_matches_cpu_adjoint(case):
    mk, ns = CASES[case]
    wl = mk()
    Jg, g = _gpu_grad(wl, ns)
    Jo, go = _oracle_grad(wl, ns)
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(case, "J %.12e vs %.12e  gradient rel L2 %.3e" % (Jg, Jo, err), flush=True)
    assert abs(Jg - Jo) <= 1e-10 * abs(Jo)
    assert err <= 1e-8


# the FP32+refine form on the cases whose boxes its kernels take (2-D lines
# of at most 32 cells): Dirichlet and pure Neumann, overlaps 0 to 3, both
# interface spaces, thin subdomains, and a full batch member
FP32_CASES = ["const_l2_dirichlet", "linear_l0", "linear_l3", "neumann_wells_l2", "beta_const",
              "no_smoothing", "thin_rows_l0", "grid64_sub4x4", "batch_member_256"]


@pytest.mark.parametrize("case", FP32_CASES)
def test_fp32_refine_adjoint_matches_cpu_adjoint(case):
    """Every local solve is refined to a componentwise backward error of
    1e-12, so the FP32+refine map stays within about 1e-10 of the FP64 map
    (measured: J within 3e-10 and the gradient within 2e-9 on the full batch
    member, which amplifies most through its five smoothing steps); bars:
    J 1e-8 and gradient 1e-7 relative, well inside the 1e-6 that the
    FP32+refine form is held to."""
    mk, ns = CASES[case]
    wl = mk()
    Jg, g = _gpu_grad(wl, ns, "fp32_refine")
    Jo, go = _oracle_grad(wl, ns)
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(case, "fp32_refine J %.12e vs %.12e  gradient rel L2 %.3e" % (Jg, Jo, err), flush=True)
    assert abs(Jg - Jo) <= 1e-8 * abs(Jo)
    assert err <= 1e-7


def test_fp32_refine_adjoint_equals_fp64_adjoint_c5():
    """Full member of the batch workload: the two precision forms' device
    gradients against each other."""
    wl = make_workload("c5")
    J64, g64 = _gpu_grad(wl, wl.nsmooth, "fp64")
    J32, g32 = _gpu_grad(wl, wl.nsmooth, "fp32_refine")
    err = np.linalg.norm(g32 - g64) / np.linalg.norm(g64)
    print("c5 member: J fp64 %.12e fp32_refine %.12e; gradient rel L2 %.3e" % (J64, J32, err), flush=True)
    assert abs(J32 - J64) <= 1e-8 * abs(J64)
    assert err <= 1e-7


def test_adjoint_matches_finite_differences_c5():
    """Full-size member of the batch workload (256 x 256, 16 x 16 subdomains,
    overlap 2, 5 smoothing steps): directional derivative of J along a random
    direction by central differences of the device forward map."""
    wl = make_workload("c5")
    J0, g = _gpu_grad(wl, wl.nsmooth)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(g.size)
    eps = 1e-4
    Jp, _ = _gpu_grad(wl.with_(logk=wl.logk + eps * v.reshape(wl.logk.shape)), wl.nsmooth)
    Jm, _ = _gpu_grad(wl.with_(logk=wl.logk - eps * v.reshape(wl.logk.shape)), wl.nsmooth)
    fd = (Jp - Jm) / (2 * eps)
    ad = float(g @ v)
    print("c5 J %.10e  directional derivative adjoint %.10e  FD %.10e  rel %.2e"
          % (J0, ad, fd, abs(ad - fd) / abs(fd)), flush=True)
    assert abs(ad - fd) <= 1e-4 * abs(fd)


def test_autograd_function_uses_the_device_adjoint():
    import torch
    import paper_2404_13811_amd as m
    wl = _small(space="linear", overlap=2)
    obs, d, fw = _weights(wl)
    lk = torch.tensor(wl.logk.ravel(), dtype=torch.float64, device="cuda", requires_grad=True)
    p, fl = m.solve_differentiable(lk, wl, nsmooth=2)
    J = 0.5 * ((p[torch.as_tensor(obs, device="cuda")] - torch.as_tensor(d, device="cuda")) ** 2).sum() \
        + (torch.as_tensor(fw.ravel(), device="cuda") * fl).sum()
    J.backward()
    _, g = _gpu_grad(wl, 2)
    assert np.allclose(lk.grad.cpu().numpy(), g, rtol=1e-12, atol=1e-14 * np.abs(g).max())


def test_autograd_function_fp32_refine():
    import torch
    import paper_2404_13811_amd as m
    wl = _small(space="const", overlap=2)
    obs, d, fw = _weights(wl)
    lk = torch.tensor(wl.logk.ravel(), dtype=torch.float64, device="cuda", requires_grad=True)
    p, fl = m.solve_differentiable(lk, wl, nsmooth=2, precision="fp32_refine")
    J = 0.5 * ((p[torch.as_tensor(obs, device="cuda")] - torch.as_tensor(d, device="cuda")) ** 2).sum() \
        + (torch.as_tensor(fw.ravel(), device="cuda") * fl).sum()
    J.backward()
    _, g = _gpu_grad(wl, 2, "fp32_refine")
    assert np.allclose(lk.grad.cpu().numpy(), g, rtol=1e-12, atol=1e-14 * np.abs(g).max())


def test_gradcheck_on_a_16x16_grid():
    """torch.autograd.gradcheck of the differentiable solve (device forward,
    device adjoint) on a 16 x 16 grid: J = misfit at 16 cells + outflow."""
    import torch
    import paper_2404_13811_amd as m
    wl = make_workload("c1", scale=4).with_(sub=(4, 4), overlap=2, beta_mode="alpha", beta_mbf=1.0,
                                             beta_smooth=1.0)
    assert tuple(wl.ncell) == (16, 16)
    obs, d, fw = _weights(wl)
    obs_t = torch.as_tensor(obs, device="cuda")
    d_t = torch.as_tensor(d, device="cuda")
    fw_t = torch.as_tensor(fw.ravel(), device="cuda")

    def J(lk):
        p, fl = m.solve_differentiable(lk, wl, nsmooth=2)
        return 0.5 * ((p[obs_t] - d_t) ** 2).sum() + (fw_t * fl).sum()

    lk = torch.tensor(wl.logk.ravel(), dtype=torch.float64, device="cuda", requires_grad=True)
    # the adjoint sums the overlapping boxes' contributions with atomic adds,
    # so two backward calls agree to rounding, not bit for bit
    assert torch.autograd.gradcheck(J, (lk,), eps=1e-6, atol=1e-7, rtol=1e-5, nondet_tol=1e-12)
