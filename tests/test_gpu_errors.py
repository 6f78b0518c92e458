"""Error reporting of the device path: a permeability that is not finite
and positive is detected by the kernels and reported by the output call
(MRCM_EINVAL); the next valid solve on the same context is clean and equal,
bit for bit, to the solve before the error."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from inputs import make_workload  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_bad_permeability_reported_then_cleared(precision):
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    wl = make_workload("c2", scale=4, overlap=2)
    good = torch.as_tensor(wl.logk.ravel(), dtype=torch.float64, device="cuda").contiguous()
    bad = good.clone()
    bad[37] = float("nan")

    def solve():
        m.build_basis(ctx)
        m.solve_interface(ctx)
        m.smooth(ctx, 2)
        p, fl = m.get_solution(ctx)
        return p.cpu().numpy(), fl.cpu().numpy()

    ctx = m.create(wl.dim, wl.ncell, wl.h)
    try:
        api.configure(ctx, wl, precision, tol=1e-12, max_refine=30)
        p0, f0 = solve()
        m.set_permeability(ctx, bad)
        with pytest.raises(m.MRCMError) as err:
            solve()
        assert err.value.status == 1  # MRCM_EINVAL
        m.set_permeability(ctx, good)
        p1, f1 = solve()
        assert np.array_equal(p0, p1) and np.array_equal(f0, f1)
    finally:
        m.destroy(ctx)


def test_forward_error_reported_by_the_adjoint_call():
    """A forward solve whose output was never read leaves its device error
    flag set; the adjoint call that follows reads it (it must not clear
    it), so the gradient of a solve with a bad permeability is refused."""
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    wl = make_workload("c5", scale=4)
    good = torch.as_tensor(wl.logk.ravel(), dtype=torch.float64, device="cuda").contiguous()
    bad = good.clone()
    bad[11] = float("nan")
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    try:
        api.configure(ctx, wl, "fp64")
        m.set_checkpointing(ctx, True)
        m.set_permeability(ctx, bad)
        m.build_basis(ctx)
        m.solve_interface(ctx)
        m.smooth(ctx, 2)
        dJdp = torch.ones(wl.ncells, dtype=torch.float64, device="cuda")
        with pytest.raises(m.MRCMError) as err:
            m.adjoint(ctx, dJdp, None)
        assert err.value.status == 1  # MRCM_EINVAL
        # the error was read: a clean solve and gradient follow
        m.set_permeability(ctx, good)
        m.build_basis(ctx)
        m.solve_interface(ctx)
        m.smooth(ctx, 2)
        g = m.adjoint(ctx, dJdp, None)
        assert bool(torch.isfinite(g).all())
    finally:
        m.destroy(ctx)
