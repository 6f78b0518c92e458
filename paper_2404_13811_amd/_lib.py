"""ctypes loader for libmrcm.so (the HIP library built from csrc/).

The library is required: there is no fallback path.  Importing this module
on a machine without the built library raises immediately.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmrcm.so")

STATUS = {0: "MRCM_OK", 1: "MRCM_EINVAL", 2: "MRCM_ENOMEM", 3: "MRCM_EDEVICE", 4: "MRCM_ESTATE",
          5: "MRCM_ENOTPD", 6: "MRCM_ENOCONV", 7: "MRCM_EINCOMPAT", 8: "MRCM_ESINGULAR"}

SYMBOLS = ("mrcm_create", "mrcm_create_batched", "mrcm_set_permeability", "mrcm_set_permeability_diag",
           "mrcm_set_source", "mrcm_set_bc",
           "mrcm_set_partition", "mrcm_set_interface_space", "mrcm_set_interface_solver",
           "mrcm_set_robin", "mrcm_set_smoothing", "mrcm_set_smoothing_persistent",
           "mrcm_set_timing", "mrcm_set_deferred_errors", "mrcm_wait", "mrcm_set_checkpointing", "mrcm_adjoint",
           "mrcm_set_precision", "mrcm_build_basis", "mrcm_solve_interface", "mrcm_smooth",
           "mrcm_get_pressure", "mrcm_get_flux", "mrcm_get_solution", "mrcm_get_coefficients", "mrcm_get_stats",
           "mrcm_get_balance", "mrcm_get_balance_static", "mrcm_rel_error", "mrcm_set_interface_check", "mrcm_last_error",
           "mrcm_destroy")


class Stats(ctypes.Structure):
    _fields_ = [("n_subdomains", ctypes.c_int), ("n_boxes", ctypes.c_int),
                ("n_unknowns", ctypes.c_int), ("band_kl", ctypes.c_int),
                ("band_ku", ctypes.c_int), ("n_local_solves", ctypes.c_int),
                ("refine_max_iters", ctypes.c_int), ("refine_max_resid", ctypes.c_double),
                ("ms_basis", ctypes.c_double), ("ms_interface", ctypes.c_double),
                ("ms_smooth", ctypes.c_double), ("bytes_factor", ctypes.c_double),
                ("ms_interface_solve", ctypes.c_double), ("interface_solver", ctypes.c_int),
                ("n_smooth_launches", ctypes.c_int), ("ms_basis_kernel", ctypes.c_double),
                ("smooth_threads", ctypes.c_int), ("smooth_graph", ctypes.c_int),
                ("ms_autotune", ctypes.c_double), ("n_smooth_phases", ctypes.c_int),
                ("smooth_persistent", ctypes.c_int), ("interface_residual", ctypes.c_double),
                ("smooth_cached", ctypes.c_int)]


class Balance(ctypes.Structure):
    _fields_ = [("mass_residual_max", ctypes.c_double), ("mass_residual_rel", ctypes.c_double),
                ("source_total", ctypes.c_double), ("outflow", ctypes.c_double * 6),
                ("outflow_total", ctypes.c_double), ("flux_jump_max", ctypes.c_double),
                ("pressure_jump_max", ctypes.c_double)]


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError("libmrcm.so is not built (%s); run __graft_entry__.build()" % LIBPATH)
    lib = ctypes.CDLL(LIBPATH)
    vp, i, d, ip = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_int)
    sig = {
        "mrcm_create": [i, ip, d, vp, ctypes.POINTER(vp)],
        "mrcm_create_batched": [i, ip, d, i, vp, ctypes.POINTER(vp)],
        "mrcm_set_permeability": [vp, vp],
        "mrcm_set_permeability_diag": [vp, vp],
        "mrcm_set_source": [vp, vp],
        "mrcm_set_bc": [vp, i, i, vp],
        "mrcm_set_partition": [vp, ip, i],
        "mrcm_set_interface_space": [vp, i],
        "mrcm_set_interface_solver": [vp, i],
        "mrcm_set_robin": [vp, i, d, d],
        "mrcm_set_smoothing": [vp, i, i],
        "mrcm_set_smoothing_persistent": [vp, i, i],
        "mrcm_set_timing": [vp, i],
        "mrcm_set_deferred_errors": [vp, i],
        "mrcm_wait": [vp],
        "mrcm_set_checkpointing": [vp, i],
        "mrcm_adjoint": [vp, vp, vp, vp],
        "mrcm_set_precision": [vp, i, d, i],
        "mrcm_build_basis": [vp],
        "mrcm_solve_interface": [vp],
        "mrcm_smooth": [vp, i],
        "mrcm_get_pressure": [vp, vp],
        "mrcm_get_flux": [vp, vp],
        "mrcm_get_solution": [vp, vp, vp],
        "mrcm_get_coefficients": [vp, vp],
        "mrcm_get_stats": [vp, ctypes.POINTER(Stats)],
        "mrcm_get_balance": [vp, vp, vp, ctypes.POINTER(Balance)],
        "mrcm_get_balance_static": [vp, vp, vp, ctypes.POINTER(Balance)],
        "mrcm_set_interface_check": [vp, d],
        "mrcm_rel_error": [vp, vp, vp, ctypes.POINTER(ctypes.c_double)],
        "mrcm_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.mrcm_last_error.argtypes = [vp]
    lib.mrcm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib
