"""The library's plan against the closed-form counts of the benchmark
workloads (M x M subdomains; 2 p unknowns per coarse interface, p = 1 for
piecewise-constant and 2 for piecewise-linear spaces in 2-D, 2 M (M - 1)
interfaces), and the local-solve count of Algorithm 1: one per seed plus
one particular problem per subdomain, then one per subdomain and smoothing
step."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from inputs import make_workload  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,overlap,expected", [("c1", None, 48), ("c2", 0, 1920), ("c2", 4, 1920),
                                                   ("c3", None, 16128), ("c5", None, 960)])
def test_plan_counts(name, overlap, expected):
    import paper_2404_13811_amd as m
    from paper_2404_13811_amd import api
    wl = make_workload(name, overlap=overlap)
    M = wl.ncell[0] // wl.sub[0]
    ctx = m.create(wl.dim, wl.ncell, wl.h)
    try:
        api.configure(ctx, wl, "fp64")
        m.build_basis(ctx)
        m.solve_interface(ctx)
        m.smooth(ctx, wl.nsmooth)
        m.get_solution(ctx)
        st = m.get_stats(ctx)
        print(name, overlap, st["n_subdomains"], st["n_unknowns"], st["n_local_solves"], flush=True)
        assert st["n_subdomains"] == M * M
        assert st["n_unknowns"] == expected
        # seeds: one unknown of X per seed (each interface function is seeded
        # from both sides), plus the particular problems and the smoothing
        assert st["n_local_solves"] == expected + M * M + wl.nsmooth * M * M
    finally:
        m.destroy(ctx)
