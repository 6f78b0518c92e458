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


_CACHE = {}


def _key(wl, nsmooth):
    import hashlib
    h = hashlib.sha256(np.ascontiguousarray(wl.logk).tobytes())
    if wl.logk_axes is not None:
        h.update(b"tensor")
        h.update(np.ascontiguousarray(wl.logk_axes).tobytes())
    h.update(np.ascontiguousarray(wl.source).tobytes())
    for v in wl.bc_value:
        h.update(np.ascontiguousarray(v).tobytes())
    return (wl.name, tuple(wl.ncell), tuple(wl.sub), wl.overlap, wl.space, wl.beta_mode,
            wl.beta_mbf, wl.beta_smooth, tuple(wl.bc_type), wl.nsmooth if nsmooth is None else nsmooth,
            h.hexdigest())


def oracle_solve(wl, nsmooth=None):
    """Oracle solve of a workload; large results are kept for the other
    tests of the session that compare against the same workload."""
    k = _key(wl, nsmooth)
    if k in _CACHE:
        return _CACHE[k]
    s = oracle_mrcm.solve(wl, nsmooth=nsmooth)
    out = (s.pressure(), s.flux().ravel(), s.X, s)
    if wl.ncells >= 256 * 256:
        _CACHE[k] = out
    return out
