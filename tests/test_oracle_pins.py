"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's formulas: each compares the oracle with
an independent route (an explicit mixed assembly, a brute-force fine solve,
a dense monolithic system, an analytic solution, a mirrored problem, a
printed table) chosen so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle breaks at least one of them.
"""
import os
import re

import numpy as np
import pytest

from inputs import make_workload
from oracle import mrcm, monolithic, rt0_mixed, tpfa
from oracle.mrcm import rel_l2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small(**kw):
    base = make_workload("c1", scale=2).with_(beta_mode="alpha", beta_mbf=1.0,
                                               beta_smooth=1.0, sub=(8, 8))
    return base.with_(**kw)


def _mrcm_o(wl):
    s = mrcm.MRCM(wl)
    s.build_basis()
    s.particular()
    s.assemble_interface()
    s.solve_interface()
    return s


# --------------------------------------------------------------- discretisation
def test_tpfa_equals_explicit_rt0_mixed_with_all_face_types():
    """Two-point flux (Section 2 remark) == RT0 mixed + trapezoid quadrature,
    on a box with Dirichlet, Neumann and Robin sides."""
    rng = np.random.default_rng(7)
    big_n = (6, 4)
    K = np.exp(rng.normal(size=big_n[::-1]))
    h = 0.25
    gbig = tpfa.Grid(big_n, h, K)
    bc_type = ("D", "D", "N", "D")
    bc_value = [rng.normal(size=4), rng.normal(size=4), rng.normal(size=6), rng.normal(size=6)]
    f = rng.normal(size=big_n[::-1])
    beta = rng.uniform(0.2, 2.0, size=4)
    lam = rng.normal(size=4)
    box = tpfa.BoxProblem(gbig, bc_type, (1, 0), (6, 4), lambda a, c, o: beta)
    p_box = box.solve(box.rhs(f=f, bc_value=bc_value, lam={0: lam}))
    # same region as a stand-alone grid, Robin on its -x side
    Ksm = K[:, 1:]
    gsm = tpfa.Grid((5, 4), h, Ksm)
    bsm = [None, bc_value[1], bc_value[2][1:], bc_value[3][1:]]
    p_mix, u_mix, faces = rt0_mixed.mixed_solve(gsm, ("N", "D", "N", "D"), bsm, f[:, 1:],
                                                robin={0: (beta, lam)})
    assert rel_l2(p_box, p_mix) < 1e-12
    # Robin velocities agree too
    u_rob = box.robin_velocity(p_box, 0, lam)
    idx = [k for k, (c, a, s, nb) in enumerate(faces) if a == 0 and s == 0 and nb < 0]
    # both are the velocity along the outward normal of the box (Section 2:
    # u.n on the boundary with n exterior), so they agree in sign as well
    assert np.allclose(u_rob, u_mix[idx], rtol=1e-11, atol=1e-12)
    assert np.abs(u_rob).max() > 1e-3


def test_fine_solution_converges_second_order_to_analytic():
    """Homogeneous problem of Section 5: p = cos(2 pi x) cos(2 pi y)."""
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        xc = (np.arange(n) + 0.5) * h
        f = 8 * np.pi ** 2 * np.outer(np.cos(2 * np.pi * xc), np.cos(2 * np.pi * xc))
        g = tpfa.Grid((n, n), h, np.ones((n, n)))
        p = tpfa.fine_solve(g, ("N",) * 4, [np.zeros(n)] * 4, f)
        ex = np.outer(np.cos(2 * np.pi * xc), np.cos(2 * np.pi * xc)).ravel()
        errs.append(np.sqrt(np.mean((p - ex) ** 2)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


def test_linear_pressure_is_reproduced_by_fine_solve():
    wl = _small(logk=np.zeros((32, 32)))
    p, _ = mrcm.fine(wl)
    xc = (np.arange(32) + 0.5) / 32
    assert np.abs(p.reshape(32, 32) - (1 - xc)[None, :]).max() < 1e-12


# --------------------------------------------------------------- Proposition 2
@pytest.mark.parametrize("overlap", [0, 1, 2])
def test_prop2_full_interface_spaces_give_fine_solution(overlap):
    wl = _small(space="fine", overlap=overlap)
    s = _mrcm_o(wl)
    pf, ff = mrcm.fine(wl)
    assert rel_l2(s.pressure(), pf) < 1e-11
    assert rel_l2(s.flux(), ff) < 1e-11


def test_prop2_pure_neumann_with_source():
    wl = make_workload("c2", scale=8).with_(space="fine", overlap=0, sub=(8, 8))
    s = _mrcm_o(wl)
    pf, ff = mrcm.fine(wl)
    assert rel_l2(s.pressure(), pf) < 1e-10
    assert rel_l2(s.flux(), ff) < 1e-10


def test_prop2_three_dimensions():
    rng = np.random.default_rng(3)
    n = (8, 8, 4)
    wl = make_workload("c4", scale=4).with_(
        ncell=n, logk=rng.normal(size=n[::-1]), source=np.zeros(n[::-1]),
        bc_value=[np.full(32, 1.0), np.zeros(32), np.zeros(32), np.zeros(32), np.zeros(64), np.zeros(64)],
        sub=(4, 4, 4), overlap=1, space="fine")
    s = _mrcm_o(wl)
    pf, ff = mrcm.fine(wl)
    assert rel_l2(s.pressure(), pf) < 1e-11
    assert rel_l2(s.flux(), ff) < 1e-11


# --------------------------------------------------------------- exactness
def test_linear_pressure_exact_with_linear_spaces_no_overlap():
    """Constant K, p = 1 - x: the exact Robin data are linear on every side,
    so they lie in the span of the piecewise-linear seeds."""
    wl = _small(logk=np.zeros((32, 32)), space="linear", overlap=0)
    s = mrcm.solve(wl, nsmooth=0)
    pf, ff = mrcm.fine(wl)
    assert rel_l2(s.pressure(), pf) < 1e-12
    assert rel_l2(s.flux(), ff) < 1e-12


def test_linear_pressure_exact_with_constant_spaces_on_strips():
    wl = _small(logk=np.zeros((32, 32)), space="const", overlap=0, sub=(8, 32))
    s = mrcm.solve(wl, nsmooth=0)
    pf, ff = mrcm.fine(wl)
    assert rel_l2(s.pressure(), pf) < 1e-12
    assert rel_l2(s.flux(), ff) < 1e-12


def test_single_subdomain_is_the_fine_solve():
    wl = _small(sub=(32, 32), overlap=0)
    s = mrcm.MRCM(wl)
    s.build_basis()
    s.particular()
    assert s.nseed == [0]
    assert rel_l2(s.part_sol[0]["p"], mrcm.fine(wl)[0]) < 1e-13


# --------------------------------------------------------------- monolithic
@pytest.mark.parametrize("space,overlap", [("const", 2), ("linear", 1), ("const", 0), ("linear", 3)])
def test_basis_route_equals_monolithic_system(space, overlap):
    s = _mrcm_o(_small(space=space, overlap=overlap))
    pm, gm, Xm = monolithic.solve_monolithic(s)
    assert rel_l2(s.pressure(), pm) < 1e-12
    assert np.abs(s.X - Xm).max() < 1e-10 * max(1.0, np.abs(Xm).max())


def test_monolithic_pure_neumann():
    wl = make_workload("c2", scale=8).with_(sub=(8, 8), overlap=2)
    s = _mrcm_o(wl)
    pm, _, _ = monolithic.solve_monolithic(s)
    assert rel_l2(s.pressure(), pm) < 1e-11


# --------------------------------------------------------------- invariances
def test_interface_and_seed_basis_choice_does_not_change_solution(monkeypatch):
    """Lambda_H^i, M_H and V_H are spaces: any basis of them gives the same
    solution (only the coefficients X change)."""
    wl = _small(space="linear", overlap=2)
    s0 = mrcm.solve(wl, nsmooth=1)
    orig = mrcm.side_family

    def mixed(space, lo, hi, side, d, window=None):
        v = orig(space, lo, hi, side, d, window)
        return [0.5 * v[0] + 1.3 * v[1], -2.0 * v[1] + 0.25 * v[0]]

    monkeypatch.setattr(mrcm, "side_family", mixed)
    s1 = mrcm.solve(wl, nsmooth=1)
    assert rel_l2(s1.pressure(), s0.pressure()) < 1e-12
    assert rel_l2(s1.flux(), s0.flux()) < 1e-12
    assert np.abs(s1.X - s0.X).max() > 1e-3


@pytest.mark.parametrize("overlap,n,nsmooth", [(0, 32, 0), (2, 32, 0), (0, 24, 2), (3, 24, 2)])
def test_mirrored_problem_gives_mirrored_solution(overlap, n, nsmooth):
    """Mirroring x swaps which subdomain of each vertical interface has the
    lower index, so a sign error in the unique-normal convention breaks it.
    With smoothing, an odd number of subdomains per axis keeps the colour
    order unchanged under the mirror (the sweep is multiplicative)."""
    rng = np.random.default_rng(11)
    wl = _small(space="linear", overlap=overlap, ncell=(n, n),
                logk=rng.normal(size=(n, n)), source=np.zeros((n, n)),
                bc_value=[np.ones(n), np.zeros(n), np.zeros(n), np.zeros(n)])
    s = mrcm.solve(wl, nsmooth=nsmooth)
    wm = wl.with_(logk=wl.logk[:, ::-1].copy(),
                  bc_value=[wl.bc_value[1], wl.bc_value[0], wl.bc_value[2][::-1].copy(),
                            wl.bc_value[3][::-1].copy()])
    sm = mrcm.solve(wm, nsmooth=nsmooth)
    p = s.pressure().reshape(n, n)
    pm = sm.pressure().reshape(n, n)
    assert np.abs(p[:, ::-1] - pm).max() < 1e-12
    F = s.flux().reshape(n, n, 4)
    Fm = sm.flux().reshape(n, n, 4)
    assert np.abs(F[:, ::-1, 0] - Fm[:, :, 1]).max() < 1e-10
    assert np.abs(F[:, ::-1, 2] - Fm[:, :, 2]).max() < 1e-10


# --------------------------------------------------------------- smoothing
@pytest.mark.parametrize("overlap", [0, 1, 2, 3])
def test_fine_solution_is_a_fixed_point_of_smoothing(overlap):
    wl = _small(overlap=overlap)
    s = _mrcm_o(wl)
    pf, ff = mrcm.fine(wl)
    s.p = pf.copy()
    for i in range(s.part.nsub):
        lo, hi = s.part.omega(i)
        for side in s.part.gamma_sides(i):
            c = s.grid.flat(tpfa.box_coords(lo, hi)[tpfa.side_local(lo, hi, side)])
            s.gflux[i][side] = ff[c, side]
    s.smooth(2)
    assert rel_l2(s.pressure(), pf) < 1e-12
    assert rel_l2(s.flux(), ff) < 1e-12


@pytest.mark.parametrize("overlap", [0, 2])
def test_smoothing_error_decreases_towards_fine_solution(overlap):
    wl = _small(overlap=overlap)
    s = mrcm.solve(wl, nsmooth=0)
    pf, ff = mrcm.fine(wl)
    errs = []
    for _ in range(6):
        errs.append((rel_l2(s.pressure(), pf), rel_l2(s.flux(), ff)))
        s.smooth(1)
    for k in range(5):
        assert errs[k + 1][0] < errs[k][0] and errs[k + 1][1] < errs[k][1]
    assert errs[-1][1] < (0.05 if overlap else 0.5) * errs[0][1]


def test_smoothing_is_reentrant():
    wl = _small(overlap=2)
    a = mrcm.solve(wl, nsmooth=0)
    a.smooth(2)
    a.smooth(1)
    b = mrcm.solve(wl, nsmooth=3)
    assert np.array_equal(a.pressure(), b.pressure())


# ------------------------------------------- smoothing with its own Robin parameter
# Algorithm 1, Step 6: when the smoothing Robin parameter differs from the one
# of the basis functions, the oversampled boxes are factored again with it
# (Section 3 item 3 allows any positive alpha); Step 7 then uses those boxes.
@pytest.mark.parametrize("overlap", [0, 2, 3])
@pytest.mark.parametrize("alpha_mbf", [1e-2, 1e2])
def test_fine_solution_is_a_fixed_point_of_smoothing_with_distinct_alpha(overlap, alpha_mbf):
    """Robin data taken from the fine solution reproduce it whatever the
    smoothing parameter, provided the box solve and the data use the same
    beta: a box built with the basis parameter but fed data formed with the
    smoothing one (or the reverse) leaves the fine solution."""
    wl = _small(overlap=overlap, beta_mbf=alpha_mbf, beta_smooth=1.0)
    s = _mrcm_o(wl)
    assert not s.same_beta
    pf, ff = mrcm.fine(wl)
    s.p = pf.copy()
    for i in range(s.part.nsub):
        lo, hi = s.part.omega(i)
        for side in s.part.gamma_sides(i):
            c = s.grid.flat(tpfa.box_coords(lo, hi)[tpfa.side_local(lo, hi, side)])
            s.gflux[i][side] = ff[c, side]
    s.smooth(2)
    assert rel_l2(s.pressure(), pf) < 1e-12
    assert rel_l2(s.flux(), ff) < 1e-12


@pytest.mark.parametrize("overlap", [0, 2])
@pytest.mark.parametrize("alpha_mbf", [1e-2, 1e2])
def test_distinct_alpha_smoothing_uses_the_smoothing_parameter_only(overlap, alpha_mbf):
    """From one and the same state, smoothing with alpha_sm = 1 gives the
    same iterates whether the basis was built with alpha_mbf = alpha_sm or
    not: Steps 6-7 depend on the smoothing parameter alone."""
    a = _mrcm_o(_small(overlap=overlap, beta_mbf=alpha_mbf, beta_smooth=1.0))
    b = _mrcm_o(_small(overlap=overlap, beta_mbf=1.0, beta_smooth=1.0))
    assert rel_l2(a.pressure(), b.pressure()) > 1e-6   # MRCM-O differs with alpha_mbf
    b.p = a.p.copy()
    b.gflux = [{q: v.copy() for q, v in fl.items()} for fl in a.gflux]
    a.smooth(2)
    b.smooth(2)
    assert rel_l2(a.pressure(), b.pressure()) < 1e-12
    assert rel_l2(a.flux(), b.flux()) < 1e-12


@pytest.mark.parametrize("alpha_mbf", [1e-2, 1e2])
def test_smoothing_error_decreases_with_alpha_sm_one(alpha_mbf):
    """Section 5's parameter study: basis functions with alpha_mbf far from
    one, smoothing with alpha_sm = 1; each step brings the solution closer
    to the fine one."""
    wl = _small(overlap=2, beta_mbf=alpha_mbf, beta_smooth=1.0)
    s = mrcm.solve(wl, nsmooth=0)
    pf, ff = mrcm.fine(wl)
    errs = []
    for _ in range(5):
        errs.append((rel_l2(s.pressure(), pf), rel_l2(s.flux(), ff)))
        s.smooth(1)
    for k in range(4):
        assert errs[k + 1][0] < errs[k][0] and errs[k + 1][1] < errs[k][1]
    assert errs[-1][1] < 0.2 * errs[0][1]


# --------------------------------------------------------------- conservation
@pytest.mark.parametrize("nsmooth", [0, 2])
def test_every_cell_balances_mass(nsmooth):
    wl = make_workload("c2", scale=8).with_(overlap=2, sub=(8, 8))
    s = mrcm.solve(wl, nsmooth=nsmooth)
    F = s.flux()
    h = wl.h
    bal = F.sum(axis=1) * h - wl.source.ravel() * h * h
    assert np.abs(bal).max() < 1e-12 * np.abs(F).max()


def test_global_conservation_after_mrcm_o():
    """Constant flux moments vanish on every interface, so the net boundary
    outflow equals the integral of the source."""
    wl = _small(overlap=2)
    s = _mrcm_o(wl)
    F = s.flux().reshape(32, 32, 4)
    h = wl.h
    out = (F[:, 0, 0].sum() + F[:, -1, 1].sum() + F[0, :, 2].sum() + F[-1, :, 3].sum()) * h
    assert abs(out) < 1e-12 * np.abs(F).max()


# --------------------------------------------------------------- Proposition 1 / Table 2
def test_prop1_dimensions_and_table2_counts():
    rows = []
    with open(os.path.join(GOLDEN, "table2_cost.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(line.split())
    M = 4
    for name, l, k, nlc, lp, ip in rows[1:]:
        l, k, nlc = int(l), int(k), int(nlc)
        space = "const" if name.startswith("OC") else "linear"
        wl = make_workload("homog").with_(overlap=l, space=space, nsmooth=k)
        s = mrcm.MRCM(wl)
        s.build_basis()
        interior = [i for i in range(s.part.nsub) if len(s.part.gamma_sides(i)) == 4][0]
        # local problems per subdomain: seeds + particular + smoothing steps
        assert s.nseed[interior] + 1 + k == nlc, name
        lo, hi = s.part.omega_hat(interior)
        assert "%dx%d" % (hi[0] - lo[0], hi[1] - lo[1]) == lp
        # printed interface size = dim M_H = dim V_H; Proposition 1: the
        # system has dim M_H + dim V_H unknowns
        coef = int(re.match(r"(\d)M\(M-1\)", ip).group(1))
        dim_MH = coef * M * (M - 1)
        assert s.offset[-1] == 2 * dim_MH, name
        s.particular()
        G, _ = s.assemble_interface()
        assert G.shape == (2 * dim_MH, 2 * dim_MH)


# --------------------------------------------------------------- Robin parameter
def test_solution_invariant_under_permeability_scaling():
    """beta = alpha H / K_H scales like 1/K, so multiplying K by a constant
    leaves the pressure unchanged and scales every velocity by it."""
    wl = _small(space="linear", overlap=2)
    s = mrcm.solve(wl, nsmooth=2)
    s2 = mrcm.solve(wl.with_(logk=wl.logk + np.log(7.0)), nsmooth=2)
    assert rel_l2(s2.pressure(), s.pressure()) < 1e-12
    assert rel_l2(s2.flux(), 7.0 * s.flux()) < 1e-12


def test_alpha_mode_with_constant_permeability_is_beta_alpha_H_over_K():
    """With constant K the harmonic mean is K itself, so alpha mode must equal
    a constant beta of alpha * (subdomain width) / K."""
    K = 3.0
    alpha = 0.7
    wl = _small(space="const", overlap=2, logk=np.full((32, 32), np.log(K)),
                beta_mbf=alpha, beta_smooth=alpha)
    s = mrcm.solve(wl, nsmooth=1)
    H = 8 * wl.h
    sc = mrcm.solve(wl.with_(beta_mode="const", beta_mbf=alpha * H / K, beta_smooth=alpha * H / K), nsmooth=1)
    assert rel_l2(s.pressure(), sc.pressure()) < 1e-13
