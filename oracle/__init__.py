"""CPU FP64 oracle for the MRCM-OS hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of the method of Zhou, Guiraldello and Pereira,
"Multiscale Mixed Methods with Improved Accuracy: The Role of Oversampling and
Smoothing" (arXiv 2404.13811).  It exists so that the HIP implementation can be
checked against something written directly from the paper.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
product library never does, and the two share no code.

Modules
-------
tpfa        fine-grid two-point-flux systems on boxes of cells (the RT0 +
            trapezoid/midpoint reduction of Section 2) and the global fine
            solve of the non-decomposed problem (Proposition 2 statement).
rt0_mixed   an explicit RT0 mixed assembly with trapezoid quadrature, kept
            only to pin ``tpfa`` (velocity and pressure unknowns, saddle form).
mrcm        partition, informed spaces / basis functions (Section 2.1 and the
            oversampling problem), particular solutions, the interface system
            (equations int_ujump / int_pjump), the MRCM-O solution and the
            smoothing steps (Section 3), following Algorithm 1's order.
monolithic  the MRCM-O variational system (equations 11d-14d) solved as one
            dense linear system, for tiny grids, to pin ``mrcm``.

Every function is FP64.  Pins live in ``tests/test_oracle_*.py``.
"""
from . import tpfa, mrcm, rt0_mixed, monolithic  # noqa: F401
