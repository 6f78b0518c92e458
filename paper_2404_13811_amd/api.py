"""Thin binding of the C ABI (argument marshalling only).

Arrays are torch tensors on the GPU, float64, contiguous; the library copies
inputs and writes outputs on the current torch stream.
"""
import ctypes
import weakref

import numpy as np
import torch

from . import _lib

SPACE = {"const": 0, "linear": 1, "fine": 2}
PRECISION = {"fp64": 0, "fp32_refine": 1}
BETA = {"alpha": 0, "const": 1}
IFACE_SOLVER = {"auto": 0, "band_lu": 1, "bcr": 2, "layered": 3}
BC = {"N": 0, "D": 1}


class MRCMError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__("%s -> %s: %s" % (fn, _lib.STATUS.get(status, status), msg))
        self.status = status


class Context:
    def __init__(self, handle, dim, ncell, nbatch=1):
        self.handle = handle
        self.dim = dim
        # cells per axis of the (stacked) grid: a batch stacks its members
        # along y
        self.ncell = tuple(ncell)
        self.nbatch = nbatch

    @property
    def ncells(self):
        n = 1
        for v in self.ncell:
            n *= v
        return n


def _check(ctx, fn, st):
    if st != 0:
        lib = _lib.load()
        msg = lib.mrcm_last_error(ctx.handle if ctx is not None else None)
        raise MRCMError(fn, st, msg.decode() if msg else "")


def _dev(t, n=None):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError("expected %d values, got %d" % (n, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


def create(dim, ncell, h, stream=None):
    lib = _lib.load()
    arr = (ctypes.c_int * 3)(*(list(ncell) + [1] * (3 - len(ncell))))
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    out = ctypes.c_void_p()
    st = lib.mrcm_create(int(dim), arr, float(h), ctypes.c_void_p(s), ctypes.byref(out))
    if st != 0:
        raise MRCMError("mrcm_create", st, "")
    return Context(out, dim, ncell)


def create_batched(dim, ncell, h, nbatch, stream=None):
    """A batch of nbatch 2-D problems on one grid (mrcm_create_batched)."""
    lib = _lib.load()
    arr = (ctypes.c_int * 3)(*(list(ncell) + [1] * (3 - len(ncell))))
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    out = ctypes.c_void_p()
    st = lib.mrcm_create_batched(int(dim), arr, float(h), int(nbatch), ctypes.c_void_p(s),
                                 ctypes.byref(out))
    if st != 0:
        raise MRCMError("mrcm_create_batched", st, "")
    return Context(out, dim, (ncell[0], ncell[1] * nbatch), nbatch)


def configure_batch(ctx, members, precision="fp64", tol=1e-12, max_refine=30, solver="auto"):
    """Pass the workload records of a batch (same grid, partition, spaces,
    Robin parameters and boundary types) through the set_* calls, member
    after member."""
    dev = "cuda"
    w0 = members[0]
    cat = lambda arrs: torch.as_tensor(np.concatenate([np.ravel(a) for a in arrs]),
                                       dtype=torch.float64, device=dev).contiguous()
    if any(w.logk_axes is not None for w in members):
        ax = [np.asarray(w.logk_axes if w.logk_axes is not None else
                         np.stack([w.logk] * w.dim)).reshape(w.dim, -1) for w in members]
        _set_k(ctx, None, np.concatenate(ax, axis=1), dev)
    else:
        set_permeability(ctx, cat([w.logk for w in members]))
    src = [w.source for w in members]
    set_source(ctx, cat(src) if any(np.any(a) for a in src) else None)
    for side, kind in enumerate(w0.bc_type):
        set_bc(ctx, side, kind, cat([w.bc_value[side] for w in members]))
    set_partition(ctx, w0.sub, w0.overlap)
    set_interface_space(ctx, w0.space)
    set_robin(ctx, w0.beta_mode, w0.beta_mbf, w0.beta_smooth)
    set_precision(ctx, precision, tol, max_refine)
    set_interface_solver(ctx, solver)


def set_permeability(ctx, logk):
    _check(ctx, "mrcm_set_permeability", _lib.load().mrcm_set_permeability(ctx.handle, _dev(logk, ctx.ncells)))


def set_permeability_diag(ctx, logk_axes):
    """Diagonal tensor: log K as dim x N values, component-major."""
    _check(ctx, "mrcm_set_permeability_diag",
           _lib.load().mrcm_set_permeability_diag(ctx.handle, _dev(logk_axes, ctx.dim * ctx.ncells)))


def _set_k(ctx, logk, logk_axes, dev):
    """log K of one workload, or of a batch's members stacked member after
    member (a tensor: each component over all members in order)."""
    if logk_axes is None:
        set_permeability(ctx, torch.as_tensor(np.ravel(logk), dtype=torch.float64, device=dev).contiguous())
    else:
        set_permeability_diag(ctx, torch.as_tensor(np.ravel(logk_axes), dtype=torch.float64,
                                                   device=dev).contiguous())


def set_source(ctx, f):
    _check(ctx, "mrcm_set_source", _lib.load().mrcm_set_source(ctx.handle, _dev(f, ctx.ncells)))


def set_bc(ctx, side, kind, values=None):
    k = BC[kind] if isinstance(kind, str) else int(kind)
    _check(ctx, "mrcm_set_bc", _lib.load().mrcm_set_bc(ctx.handle, int(side), k, _dev(values)))


def set_partition(ctx, sub, overlap):
    arr = (ctypes.c_int * 3)(*(list(sub) + [1] * (3 - len(sub))))
    _check(ctx, "mrcm_set_partition", _lib.load().mrcm_set_partition(ctx.handle, arr, int(overlap)))


def set_interface_space(ctx, space):
    s = SPACE[space] if isinstance(space, str) else int(space)
    _check(ctx, "mrcm_set_interface_space", _lib.load().mrcm_set_interface_space(ctx.handle, s))


def set_interface_solver(ctx, solver):
    v = IFACE_SOLVER[solver] if isinstance(solver, str) else int(solver)
    _check(ctx, "mrcm_set_interface_solver", _lib.load().mrcm_set_interface_solver(ctx.handle, v))


def set_smoothing(ctx, use_graph=True, threads_per_box=0):
    _check(ctx, "mrcm_set_smoothing",
           _lib.load().mrcm_set_smoothing(ctx.handle, int(bool(use_graph)), int(threads_per_box)))


def set_smoothing_persistent(ctx, on=True, max_groups=0):
    _check(ctx, "mrcm_set_smoothing_persistent",
           _lib.load().mrcm_set_smoothing_persistent(ctx.handle, int(bool(on)), int(max_groups)))


def set_interface_check(ctx, tol=1e-5):
    """Largest accepted componentwise backward error of the interface solve
    (tol <= 0: no check)."""
    _check(ctx, "mrcm_set_interface_check", _lib.load().mrcm_set_interface_check(ctx.handle, float(tol)))


def set_timing(ctx, on=True):
    _check(ctx, "mrcm_set_timing", _lib.load().mrcm_set_timing(ctx.handle, int(bool(on))))


def set_deferred_errors(ctx, on=True):
    """Calls stop synchronising to read device errors; ``wait`` reads them."""
    _check(ctx, "mrcm_set_deferred_errors",
           _lib.load().mrcm_set_deferred_errors(ctx.handle, int(bool(on))))


def wait(ctx):
    """Synchronise the context's stream and raise on any device-side error."""
    _check(ctx, "mrcm_wait", _lib.load().mrcm_wait(ctx.handle))


def set_robin(ctx, mode, mbf, smooth_value):
    m = BETA[mode] if isinstance(mode, str) else int(mode)
    _check(ctx, "mrcm_set_robin", _lib.load().mrcm_set_robin(ctx.handle, m, float(mbf), float(smooth_value)))


def set_precision(ctx, precision, tol=1e-12, max_refine=30):
    p = PRECISION[precision] if isinstance(precision, str) else int(precision)
    _check(ctx, "mrcm_set_precision", _lib.load().mrcm_set_precision(ctx.handle, p, float(tol), int(max_refine)))


def build_basis(ctx):
    _check(ctx, "mrcm_build_basis", _lib.load().mrcm_build_basis(ctx.handle))


def solve_interface(ctx):
    _check(ctx, "mrcm_solve_interface", _lib.load().mrcm_solve_interface(ctx.handle))


def smooth(ctx, nsteps):
    _check(ctx, "mrcm_smooth", _lib.load().mrcm_smooth(ctx.handle, int(nsteps)))


def get_pressure(ctx, out=None):
    if out is None:
        out = torch.empty(ctx.ncells, dtype=torch.float64, device="cuda")
    _check(ctx, "mrcm_get_pressure", _lib.load().mrcm_get_pressure(ctx.handle, _dev(out, ctx.ncells)))
    return out


def get_flux(ctx, out=None):
    n = ctx.ncells * 2 * ctx.dim
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device="cuda")
    _check(ctx, "mrcm_get_flux", _lib.load().mrcm_get_flux(ctx.handle, _dev(out, n)))
    return out


def get_solution(ctx, p_out=None, flux_out=None):
    """Pressure and face velocities with one stream synchronisation."""
    n = ctx.ncells
    if p_out is None:
        p_out = torch.empty(n, dtype=torch.float64, device="cuda")
    if flux_out is None:
        flux_out = torch.empty(n * 2 * ctx.dim, dtype=torch.float64, device="cuda")
    _check(ctx, "mrcm_get_solution",
           _lib.load().mrcm_get_solution(ctx.handle, _dev(p_out, n), _dev(flux_out, n * 2 * ctx.dim)))
    return p_out, flux_out


def get_stats(ctx):
    st = _lib.Stats()
    _check(ctx, "mrcm_get_stats", _lib.load().mrcm_get_stats(ctx.handle, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in st._fields_}


def get_balance(ctx, cell_residual=False, jumps=False, static=False):
    """Mass balance, boundary outflow and interface jump measures of the
    current solution (mrcm_get_balance, or mrcm_get_balance_static with
    static=True); optionally the per-cell residuals and the per-row jump
    moments as device tensors (allocated here, outside the C call)."""
    n = ctx.ncells
    res = torch.empty(n, dtype=torch.float64, device="cuda") if cell_residual else None
    nrow = get_stats(ctx)["n_unknowns"] if jumps else 0
    mom = torch.empty(max(nrow, 1), dtype=torch.float64, device="cuda") if jumps else None
    b = _lib.Balance()
    fn = "mrcm_get_balance_static" if static else "mrcm_get_balance"
    _check(ctx, fn, getattr(_lib.load(), fn)(
        ctx.handle, _dev(res) if res is not None else None, _dev(mom) if mom is not None else None,
        ctypes.byref(b)))
    out = {k: getattr(b, k) for k, _ in b._fields_}
    out["outflow"] = list(b.outflow)
    if res is not None:
        out["cell_residual"] = res
    if mom is not None:
        out["jumps"] = mom[:nrow]
    return out


def get_balance_static(ctx, cell_residual=False, jumps=False):
    """mrcm_get_balance_static: get_balance with no allocation in the call."""
    return get_balance(ctx, cell_residual, jumps, static=True)


def rel_error(ctx, p_ref=None, flux_ref=None):
    """Relative L2 distances (pressure, flux) of the current outputs from
    device reference arrays (mrcm_rel_error)."""
    o = (ctypes.c_double * 2)()
    n = ctx.ncells
    _check(ctx, "mrcm_rel_error", _lib.load().mrcm_rel_error(
        ctx.handle, _dev(p_ref, n) if p_ref is not None else None,
        _dev(flux_ref, n * 2 * ctx.dim) if flux_ref is not None else None, o))
    return o[0], o[1]


def set_checkpointing(ctx, on=True):
    _check(ctx, "mrcm_set_checkpointing", _lib.load().mrcm_set_checkpointing(ctx.handle, int(bool(on))))


def adjoint(ctx, dJdp=None, dJdflux=None, out=None):
    """dJ/dlog K (device tensor) for the given output adjoints (mrcm_adjoint)."""
    n = ctx.ncells
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device="cuda")
    gp = None if dJdp is None else dJdp.detach().to(device="cuda", dtype=torch.float64).contiguous()
    gf = None if dJdflux is None else dJdflux.detach().to(device="cuda", dtype=torch.float64).contiguous()
    _check(ctx, "mrcm_adjoint", _lib.load().mrcm_adjoint(
        ctx.handle, _dev(gp, n) if gp is not None else None,
        _dev(gf, n * 2 * ctx.dim) if gf is not None else None, _dev(out, n)))
    return out


class _SolveFn(torch.autograd.Function):
    """(pressure, flux) = MRCM-OS(log K); backward = mrcm_adjoint."""

    @staticmethod
    def forward(actx, logk, wl, nsmooth, precision):
        ctx = create(wl.dim, wl.ncell, wl.h)
        try:
            configure(ctx, wl, precision)
            set_permeability(ctx, logk.detach().to(device="cuda", dtype=torch.float64).contiguous())
            set_checkpointing(ctx, True)
            build_basis(ctx)
            solve_interface(ctx)
            smooth(ctx, wl.nsmooth if nsmooth is None else nsmooth)
            p = get_pressure(ctx)
            fl = get_flux(ctx)
        except Exception:
            destroy(ctx)
            raise
        # the context keeps the factors and checkpoints every backward call
        # reads (the graph may be differentiated more than once); it is
        # released with the graph, not at interpreter exit
        actx.mrcm = ctx
        fin = weakref.finalize(ctx, _lib.load().mrcm_destroy, ctx.handle)
        fin.atexit = False
        return p, fl

    @staticmethod
    def backward(actx, gp, gfl):
        g = adjoint(actx.mrcm, gp, gfl)
        return g, None, None, None


def solve_differentiable(logk, wl, nsmooth=None, precision="fp64"):
    """MRCM-OS pressure and face velocities as differentiable functions of
    log K (a CUDA float64 tensor of N values); the gradient runs the device
    adjoint in the forward solve's precision ("fp64" or "fp32_refine").  The
    workload record supplies everything else."""
    return _SolveFn.apply(logk, wl, nsmooth, precision)


def get_coefficients(ctx, out=None):
    n = get_stats(ctx)["n_unknowns"]
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
    _check(ctx, "mrcm_get_coefficients", _lib.load().mrcm_get_coefficients(ctx.handle, _dev(out)))
    return out[:n]


def destroy(ctx):
    if ctx.handle:
        _lib.load().mrcm_destroy(ctx.handle)
        ctx.handle = None


def configure(ctx, wl, precision="fp64", tol=1e-12, max_refine=30, solver="auto"):
    """Pass a workload record (inputs.Workload) through the set_* calls."""
    dev = "cuda"
    _set_k(ctx, wl.logk, wl.logk_axes, dev)
    src = wl.source.ravel()
    set_source(ctx, torch.as_tensor(src, dtype=torch.float64, device=dev).contiguous() if src.any() else None)
    for side, (kind, vals) in enumerate(zip(wl.bc_type, wl.bc_value)):
        set_bc(ctx, side, kind, torch.as_tensor(vals, dtype=torch.float64, device=dev).contiguous())
    set_partition(ctx, wl.sub, wl.overlap)
    set_interface_space(ctx, wl.space)
    set_robin(ctx, wl.beta_mode, wl.beta_mbf, wl.beta_smooth)
    set_precision(ctx, precision, tol, max_refine)
    set_interface_solver(ctx, solver)


def solve_workload(wl, precision="fp64", nsmooth=None, tol=1e-12, max_refine=30, keep=False,
                   solver="auto", check=None):
    """Full MRCM-OS solve of a workload; returns (pressure, flux[, ctx]).
    check: tolerance of the interface solve's check (None: the default)."""
    ctx = create(wl.dim, wl.ncell, wl.h)
    try:
        configure(ctx, wl, precision, tol, max_refine, solver)
        if check is not None:
            set_interface_check(ctx, check)
        build_basis(ctx)
        solve_interface(ctx)
        smooth(ctx, wl.nsmooth if nsmooth is None else nsmooth)
        p = get_pressure(ctx)
        fl = get_flux(ctx)
    except Exception:
        destroy(ctx)
        raise
    if keep:
        return p, fl, ctx
    destroy(ctx)
    return p, fl
