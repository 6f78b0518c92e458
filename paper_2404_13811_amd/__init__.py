"""MI355X-native MRCM-OS hot path (arXiv 2404.13811).

Python binding of the C ABI declared in ``include/mrcm.h``: one function per
C entry point with the same name, marshalling torch device tensors to raw
pointers.  Every numerical step runs in the HIP kernels of ``libmrcm.so``;
there is no CPU path.
"""
from .api import (MRCMError, Context, create, set_permeability, set_permeability_diag, set_source, set_bc,
                  set_partition, set_interface_space, set_interface_solver, set_robin, set_smoothing, set_smoothing_persistent, set_timing, set_deferred_errors, wait, set_precision, build_basis,
                  solve_interface, smooth, get_pressure, get_flux, get_solution, get_coefficients, get_stats,
                  destroy, solve_workload, SPACE, PRECISION, IFACE_SOLVER,
                  set_checkpointing, adjoint, solve_differentiable, get_balance, rel_error,
                  set_interface_check, get_balance_static, create_batched, configure_batch)

__all__ = ["MRCMError", "Context", "create", "set_permeability", "set_permeability_diag", "set_source", "set_bc",
           "set_partition", "set_interface_space", "set_interface_solver", "set_robin", "set_smoothing", "set_smoothing_persistent", "set_timing", "set_deferred_errors", "wait", "set_precision", "build_basis",
           "solve_interface", "smooth", "get_pressure", "get_flux", "get_solution", "get_coefficients",
           "get_stats", "destroy", "solve_workload", "SPACE", "PRECISION", "IFACE_SOLVER",
           "set_checkpointing", "adjoint", "solve_differentiable", "get_balance", "rel_error",
           "set_interface_check", "get_balance_static", "create_batched", "configure_batch"]
