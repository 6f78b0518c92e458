"""Pins of the CPU oracle for a diagonal permeability tensor (Section 2: K
is a symmetric positive definite tensor; on a Cartesian grid a diagonal
one enters each face through the entry of the face's axis).

Independent routes: the explicit mixed (RT0) assembly with the tensor's
inverse in its mass matrix, a one-dimensional series-resistance recursion,
an affine pressure that the piecewise-linear interface spaces contain, the
full-space interface proposition (Prop. 2), and the problem mirrored across
the diagonal.  Each cross-direction entry is random, so using the wrong
axis's entry anywhere breaks one of them.
"""
import numpy as np
import pytest

from inputs import make_workload
from inputs.workloads import Workload
from oracle import mrcm, rt0_mixed, tpfa
from oracle.mrcm import rel_l2


def test_tpfa_equals_rt0_mixed_with_a_diagonal_tensor():
    """Two-point flux == RT0 mixed with trapezoid quadrature (mass matrix
    1/K_a for the fluxes along axis a), with Dirichlet, Neumann and Robin
    sides and independent random entries per axis."""
    rng = np.random.default_rng(11)
    n = (6, 4)
    K = np.exp(rng.normal(size=(2,) + n[::-1]))
    h = 0.25
    g = tpfa.Grid(n, h, K)
    assert not g.isotropic
    bc_type = ("D", "D", "N", "D")
    bc_value = [rng.normal(size=4), rng.normal(size=4), rng.normal(size=6), rng.normal(size=6)]
    f = rng.normal(size=n[::-1])
    beta = rng.uniform(0.2, 2.0, size=4)
    lam = rng.normal(size=4)
    box = tpfa.BoxProblem(g, bc_type, (1, 0), (6, 4), lambda a, c, o: beta)
    p_box = box.solve(box.rhs(f=f, bc_value=bc_value, lam={0: lam}))
    gsm = tpfa.Grid((5, 4), h, K[:, :, 1:])
    bsm = [None, bc_value[1], bc_value[2][1:], bc_value[3][1:]]
    p_mix, u_mix, faces = rt0_mixed.mixed_solve(gsm, ("N", "D", "N", "D"), bsm, f[:, 1:],
                                                robin={0: (beta, lam)})
    assert rel_l2(p_box, p_mix) < 1e-12
    u_rob = box.robin_velocity(p_box, 0, lam)
    idx = [k for k, (c, a, s, nb) in enumerate(faces) if a == 0 and s == 0 and nb < 0]
    assert np.allclose(u_rob, u_mix[idx], rtol=1e-11, atol=1e-12)


def _series(kflow, h, pl, pr):
    """Cell pressures and the face velocity of 1-D flow through cells of
    permeability kflow between pressures pl and pr (half-cell resistances
    h / 2K at the ends, h / K_H between cells)."""
    kh = 2.0 * kflow[:-1] * kflow[1:] / (kflow[:-1] + kflow[1:])
    R = h / (2.0 * kflow[0]) + np.sum(h / kh) + h / (2.0 * kflow[-1])
    q = (pl - pr) / R
    p = np.empty(kflow.size)
    p[0] = pl - q * h / (2.0 * kflow[0])
    for i in range(kflow.size - 1):
        p[i + 1] = p[i] - q * h / kh[i]
    return p, q


def _flow_workload(ncell, axis, kflow, cross, space="linear", overlap=2, sub=None):
    """Dirichlet 1 / 0 on the two sides normal to `axis`, no flow through
    the others; K along `axis` = kflow (a function of that coordinate), the
    other entries `cross` (random per cell)."""
    d = len(ncell)
    shape = tuple(ncell[::-1])
    kf = np.broadcast_to(kflow.reshape([-1 if b == d - 1 - axis else 1 for b in range(d)]), shape)
    ax = np.array([np.log(kf) if a == axis else np.log(cross[a]) for a in range(d)])
    types, vals = [], []
    for side in range(2 * d):
        a = side // 2
        nf = int(np.prod([ncell[b] for b in range(d) if b != a]))
        if a == axis:
            types.append("D")
            vals.append(np.full(nf, 1.0 if side % 2 == 0 else 0.0))
        else:
            types.append("N")
            vals.append(np.zeros(nf))
    h = 1.0 / ncell[0]
    sub = sub or tuple(4 for _ in range(d))
    return Workload("tensor_flow", d, tuple(ncell), h, ax[0], np.zeros(shape), tuple(types), vals,
                    sub, overlap, space, "alpha", 1.0, 1.0, 1, logk_axes=ax)


@pytest.mark.parametrize("ncell,axis", [((16, 12), 0), ((12, 16), 1), ((8, 8, 12), 2)])
def test_one_dimensional_flow_follows_the_series_resistance(ncell, axis):
    """Flow along one axis through layers across it: the fine solution is
    the 1-D series-resistance profile whatever the other entries are, and
    no velocity crosses the other faces."""
    rng = np.random.default_rng(5 + axis)
    d = len(ncell)
    kflow = np.exp(rng.normal(size=ncell[axis]))
    cross = [np.exp(rng.normal(size=ncell[::-1])) for _ in range(d)]
    wl = _flow_workload(ncell, axis, kflow, cross)
    p, fl = mrcm.fine(wl)
    pe, q = _series(kflow, wl.h, 1.0, 0.0)
    coord = np.indices(ncell[::-1])[d - 1 - axis].ravel()
    assert np.abs(p - pe[coord]).max() < 1e-12
    # velocities: +axis faces carry q, faces normal to the other axes none
    assert np.allclose(fl[:, 2 * axis + 1], q, rtol=1e-11)
    for a in range(d):
        if a != axis:
            assert np.abs(fl[:, 2 * a:2 * a + 2]).max() < 1e-11


@pytest.mark.parametrize("ncell,axis", [((16, 16), 0), ((16, 16), 1), ((8, 8, 12), 2)])
def test_mrcm_os_is_exact_for_an_affine_pressure(ncell, axis):
    """Constant K along the flow, random entries across it: the pressure is
    affine along the flow axis, so its traces on every interface lie in
    the piecewise-linear interface spaces; without oversampling (l = 0) the
    boxes are the subdomains, the exact solution is a combination of the
    basis functions and the particular solution, and MRCM-O returns it to
    rounding (a smoothing step keeps it).  With oversampling the seeds live
    on the larger boxes' sides and the method is not exact even for scalar
    constant K (about 1e-2 here), so l = 0 is the pin."""
    overlap = 0
    rng = np.random.default_rng(21 + axis)
    d = len(ncell)
    kflow = np.full(ncell[axis], 2.5)
    cross = [np.exp(2.0 * rng.normal(size=ncell[::-1])) for _ in range(d)]
    wl = _flow_workload(ncell, axis, kflow, cross, space="linear", overlap=overlap)
    s = mrcm.solve(wl, nsmooth=1)
    pe, q = _series(kflow, wl.h, 1.0, 0.0)
    coord = np.indices(ncell[::-1])[d - 1 - axis].ravel()
    assert np.abs(s.pressure() - pe[coord]).max() < 1e-10
    fl = s.flux()
    assert np.allclose(fl[:, 2 * axis + 1], q, rtol=1e-9)


@pytest.mark.parametrize("overlap", [0, 2])
def test_prop2_full_spaces_with_a_tensor(overlap):
    """Prop. 2 holds for the discrete problem whatever K is: with the full
    interface spaces MRCM-O is the fine solution."""
    rng = np.random.default_rng(3)
    base = make_workload("c1", scale=2).with_(sub=(8, 8), beta_mode="alpha", beta_mbf=1.0,
                                               beta_smooth=1.0)
    wl = base.with_tensor([0.0, rng.normal(size=base.logk.shape)]).with_(space="fine", overlap=overlap)
    s = mrcm.MRCM(wl)
    s.build_basis()
    s.particular()
    s.assemble_interface()
    s.solve_interface()
    pf, ff = mrcm.fine(wl)
    assert rel_l2(s.pressure(), pf) < 1e-11
    assert rel_l2(s.flux(), ff) < 1e-11


def test_equal_entries_reproduce_the_scalar_oracle():
    wl = make_workload("c1", scale=2).with_(sub=(8, 8))
    a = mrcm.solve(wl, nsmooth=2)
    b = mrcm.solve(wl.with_tensor([0.0, 0.0]), nsmooth=2)
    assert np.array_equal(a.pressure(), b.pressure())
    assert np.array_equal(a.flux(), b.flux())


def test_mirrored_tensor_problem():
    """Transposing the grid swaps the axes: (K_x, K_y) becomes (K_y, K_x) on
    the transposed cells, the x sides' conditions become the y sides', and
    the MRCM-O solution is the transposed one (velocities with their sides
    swapped).  The smoothing sweeps are left out: transposing exchanges two
    colours, so their order, and with it the smoothed iterate, changes."""
    rng = np.random.default_rng(8)
    n = 32
    base = make_workload("c1", scale=2).with_(sub=(8, 8), space="linear", overlap=2)
    ky = base.logk + rng.normal(size=base.logk.shape)
    wl = base.with_(logk_axes=np.stack([base.logk, ky]))
    # transposed: new x = old y
    ax_t = np.stack([ky.T.copy(), base.logk.T.copy()])
    bt = (base.bc_type[2], base.bc_type[3], base.bc_type[0], base.bc_type[1])
    bv = [base.bc_value[2], base.bc_value[3], base.bc_value[0], base.bc_value[1]]
    wt = base.with_(logk=ax_t[0], logk_axes=ax_t, bc_type=bt, bc_value=bv,
                    source=base.source.T.copy())
    a = mrcm.solve(wl, nsmooth=0)
    b = mrcm.solve(wt, nsmooth=0)
    pa = a.pressure().reshape(n, n)
    pb = b.pressure().reshape(n, n)
    assert np.allclose(pa, pb.T, rtol=1e-11, atol=1e-13)
    fa = a.flux().reshape(n, n, 4)
    fb = b.flux().reshape(n, n, 4).transpose(1, 0, 2)[:, :, [2, 3, 0, 1]]
    assert np.allclose(fa, fb, rtol=1e-10, atol=1e-12)
    # and the tensor matters: the scalar problem differs
    c = mrcm.solve(base, nsmooth=0)
    assert rel_l2(c.pressure(), a.pressure()) > 1e-3
