"""Status codes of the C ABI: calls out of order report MRCM_ESTATE, bad
arguments MRCM_EINVAL, and neither leaves the context unusable (a full
solve afterwards gives the result of a fresh context, bit for bit)."""
import ctypes
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from inputs import make_workload  # noqa: E402

pytestmark = pytest.mark.gpu

EINVAL, ESTATE = 1, 4


def test_call_order_and_arguments():
    import torch
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import _lib, api
    lib = _lib.load()
    wl = make_workload("c1")
    ref_p, ref_f = m.solve_workload(wl, precision="fp64", solver="bcr")
    ref_p, ref_f = ref_p.cpu().numpy(), ref_f.cpu().numpy()
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    h = ctx.handle
    try:
        # nothing set yet
        assert lib.mrcm_build_basis(h) == ESTATE
        assert lib.mrcm_solve_interface(h) == ESTATE
        assert lib.mrcm_smooth(h, 1) == ESTATE
        out = torch.empty(wl.ncells, dtype=torch.float64, device="cuda")
        assert lib.mrcm_get_pressure(h, ctypes.c_void_p(out.data_ptr())) == ESTATE
        # bad arguments
        assert lib.mrcm_set_permeability(h, None) == EINVAL
        bad_sub = (ctypes.c_int * 2)(7, 7)  # 64 is not a multiple of 7
        assert lib.mrcm_set_partition(h, bad_sub, 2) == EINVAL
        assert lib.mrcm_wait(None) == EINVAL
        api.configure(ctx, wl, "fp64", solver="bcr")
        # basis built, interface not solved
        assert lib.mrcm_build_basis(h) == 0
        assert lib.mrcm_smooth(h, 1) == ESTATE
        assert lib.mrcm_get_pressure(h, ctypes.c_void_p(out.data_ptr())) == ESTATE
        assert lib.mrcm_solve_interface(h) == 0
        # outputs need a destination; the adjoint needs checkpoints
        assert lib.mrcm_get_pressure(h, None) == EINVAL
        g = torch.empty(wl.ncells, dtype=torch.float64, device="cuda")
        assert lib.mrcm_smooth(h, wl.nsmooth) == 0
        assert lib.mrcm_adjoint(h, ctypes.c_void_p(out.data_ptr()), None,
                                ctypes.c_void_p(g.data_ptr())) == ESTATE
        p, fl = m.get_solution(ctx)
        assert np.array_equal(p.cpu().numpy(), ref_p)
        assert np.array_equal(fl.cpu().numpy(), ref_f)
        assert lib.mrcm_last_error(h)  # the last failure left a message
    finally:
        m.destroy(ctx)
