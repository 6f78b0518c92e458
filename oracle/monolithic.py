"""MRCM-O as one dense linear system (oracle pin, test-only, tiny grids).

Equations eq11d-eq14d are assembled directly in the unknowns
(p^i on every Omega_i, X_i^k) without the split into particular and basis
parts (eq:addu, eq:addp) or the superposition eq:uhatphat:

* per subdomain, the local Robin problem on Omega_i with data
  ``lambda^i = sum_k X_i^k phi_i^k`` (eq11d-eq12d in two-point-flux form);
* per coarse interface and test function, flux continuity (eq13d):
  ``sum_e |e| M (u^i + u^j) = 0`` with ``u^i = T^R (p^i_c - lambda^i) / |e|``;
* pressure continuity (eq14d): ``sum_e |e| V (beta u^i + lambda^i)`` with sign
  +1 for the lower-indexed subdomain and -1 for the other.

The informed functions phi_i^k are taken from ``mrcm.MRCM.build_basis`` (they
define the space Lambda_H^i); everything downstream of them is independent of
the basis-function route.
"""
import numpy as np

from .tpfa import BoxProblem, box_coords


def solve_monolithic(solver):
    """``solver`` is an ``mrcm.MRCM`` after ``build_basis``.  Returns the
    global pressure and the per-subdomain Gamma fluxes."""
    g, part = solver.grid, solver.part
    offs_p = [0]
    boxes = []
    for i in range(part.nsub):
        lo, hi = part.omega(i)
        box = BoxProblem(g, solver.bc_type, lo, hi, solver.beta_mbf)
        boxes.append(box)
        offs_p.append(offs_p[-1] + box.nloc)
    nP = offs_p[-1]
    nX = int(solver.offset[-1])
    n = nP + nX
    Kmat = np.zeros((n, n))
    rhs = np.zeros(n)

    def lam_coeffs(i, side):
        # lambda^i on this side as a matrix (faces x seeds of i)
        return np.stack([solver.mbf[i]["traces"][k][side]["phi"] for k in range(solver.nseed[i])], axis=1)

    for i, box in enumerate(boxes):
        o = offs_p[i]
        Kmat[o:o + box.nloc, o:o + box.nloc] = box.A.toarray()
        rhs[o:o + box.nloc] = box.rhs(f=solver.f, bc_value=solver.bc_value)
        for side, e in box.robin.items():
            L = lam_coeffs(i, side)
            for r, loc in enumerate(e["local"]):
                Kmat[o + loc, nP + solver.offset[i]: nP + solver.offset[i + 1]] -= e["TR"][r] * L[r]
    row = nP
    first_flux = None
    for (i, a, j) in part.interfaces():
        qi, qj = 2 * a + 1, 2 * a
        fam = solver.interface_family(i, qi)
        for kind in ("flux", "pressure"):
            for mu in fam:
                w = g.area * mu
                for sub, q, sg in ((i, qi, 1.0), (j, qj, 1.0 if kind == "flux" else -1.0)):
                    e = boxes[sub].robin[q]
                    L = lam_coeffs(sub, q)
                    TRa = e["TR"] / g.area
                    ploc = offs_p[sub] + e["local"]
                    xs = slice(nP + solver.offset[sub], nP + solver.offset[sub + 1])
                    if kind == "flux":
                        # u = TR/|e| (p_c - lambda)
                        Kmat[row, ploc] += sg * w * TRa
                        Kmat[row, xs] += -sg * (w * TRa) @ L
                    else:
                        # beta u + lambda
                        bt = e["beta"]
                        Kmat[row, ploc] += sg * w * bt * TRa
                        Kmat[row, xs] += sg * (w @ (L - (bt * TRa)[:, None] * L) + 0.0)
                if kind == "flux" and first_flux is None:
                    first_flux = row
                row += 1
    assert row == n
    if solver.neumann:
        Kmat[first_flux, :] = 0.0
        Kmat[first_flux, nP] = 1.0
        rhs[first_flux] = 0.0
    sol = np.linalg.solve(Kmat, rhs)
    p = np.zeros(g.ncells)
    gflux = []
    X = sol[nP:]
    for i, box in enumerate(boxes):
        pi = sol[offs_p[i]:offs_p[i + 1]]
        p[box.gidx] = pi
        fl = {}
        for side, e in box.robin.items():
            lam = lam_coeffs(i, side) @ X[solver.offset[i]:solver.offset[i + 1]]
            fl[side] = e["TR"] * (pi[e["local"]] - lam) / g.area
        gflux.append(fl)
    if solver.neumann:
        p = p - p.mean()
    return p, gflux, X
