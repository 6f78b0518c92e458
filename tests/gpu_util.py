"""Helpers shared by the GPU tests (no numerical method code)."""
import numpy as np
import torch

import paper_2404_13811_amd as m
from oracle import mrcm as oracle_mrcm


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_solve(wl, precision="fp64", nsmooth=None, **kw):
    p, fl, ctx = m.solve_workload(wl, precision=precision, nsmooth=nsmooth, keep=True, **kw)
    torch.cuda.synchronize()
    X = m.get_coefficients(ctx).cpu().numpy()
    st = m.get_stats(ctx)
    m.destroy(ctx)
    return p.cpu().numpy(), fl.cpu().numpy(), X, st


def oracle_solve(wl, nsmooth=None):
    s = oracle_mrcm.solve(wl, nsmooth=nsmooth)
    return s.pressure(), s.flux().ravel(), s.X, s
