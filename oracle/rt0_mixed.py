"""Explicit lowest-order Raviart-Thomas mixed system (oracle pin, test-only).

Used only to pin ``tpfa``: it assembles the saddle-point form of equations
eq1a-eq1d (velocity unknowns on faces, pressure unknowns in cells) with the
RT0 basis on each Cartesian cell and evaluates the velocity mass matrix with
the tensor-product trapezoid rule (vertex values), as the paper prescribes for
the cell-centred equivalence (Section 2, remark on midpoint/trapezoid rules).
Robin faces contribute (beta u.n, v.n) on the face, Dirichlet faces the
boundary pressure term, Neumann faces fix the face velocity.  Dense and tiny.
"""
import itertools
import numpy as np


def _rt0_basis_at(x, a, s, h):
    """RT0 basis function of the cell [0, h]^d for face (axis a, side s),
    normalised to unit outward normal component on that face, evaluated at
    point x: only its a-component is non-zero, linear in x_a."""
    return (x[a] / h) if s == 1 else -(1.0 - x[a] / h)


def mixed_solve(grid, bc_type, bc_value, f, robin=None):
    """Solve the mixed RT0 system on the whole grid; ``robin`` optionally maps
    a boundary side to (beta per face, lam per face), overriding bc_type.

    Returns (p per cell, u per unique face in the order of ``faces``, faces)
    where faces is a list of (cell, side) with the normal along +axis for
    interior faces (owned by the lower cell) and outward on the boundary."""
    d, h, n = grid.d, grid.h, grid.n
    N = grid.ncells
    co = grid.coords(np.arange(N))
    faces = []
    fid = {}
    for c in range(N):
        for a in range(d):
            for s in (0, 1):
                nb = co[c].copy()
                nb[a] += 1 if s else -1
                inside = 0 <= nb[a] < n[a]
                if inside and s == 0:
                    continue  # owned by the lower cell
                fid[(c, a, s)] = len(faces)
                if inside:
                    fid[(int(grid.flat(nb)), a, 0)] = len(faces)
                faces.append((c, a, s, int(grid.flat(nb)) if inside else -1))
    nf = len(faces)
    # trapezoid rule on the reference cell: vertices with weight h^d / 2^d
    verts = [np.array(v, dtype=float) * h for v in itertools.product((0, 1), repeat=d)]
    wq = h ** d / 2 ** d
    Mm = np.zeros((nf, nf))
    B = np.zeros((N, nf))
    rhs_u = np.zeros(nf)
    rhs_p = np.asarray(f).ravel() * h ** d
    for c in range(N):
        loc = []
        for a in range(d):
            for s in (0, 1):
                fi = fid[(c, a, s)]
                # sign of this cell's outward normal relative to the face's unknown
                own = faces[fi][0] == c and faces[fi][1] == a and faces[fi][2] == s
                sg = 1.0 if own or faces[fi][3] < 0 else -1.0
                loc.append((fi, a, s, sg))
        for (fi, a, s, sg) in loc:
            for (fj, b, t, sg2) in loc:
                if a != b:
                    continue
                val = 0.0
                for x in verts:
                    val += wq * _rt0_basis_at(x, a, s, h) * _rt0_basis_at(x, b, t, h)
                Mm[fi, fj] += val * sg * sg2 / grid.k(c, a)
            # divergence of the basis: outward flux |e| through its own face
            B[c, fi] += sg * grid.area
    robin = robin or {}
    fixed = {}
    for fi, (c, a, s, nb) in enumerate(faces):
        if nb >= 0:
            continue
        side = 2 * a + s
        from .tpfa import boundary_face_index
        face = int(boundary_face_index(grid, co[c:c + 1], side)[0])
        if side in robin:
            beta, lam = robin[side]
            Mm[fi, fi] += beta[face] * grid.area
            rhs_u[fi] -= lam[face] * grid.area
        elif bc_type[side] == "D":
            rhs_u[fi] -= bc_value[side][face] * grid.area
        else:
            fixed[fi] = bc_value[side][face]
    # saddle system [[M, -B^T], [B, 0]] [u; p] = [rhs_u; rhs_p]
    K = np.zeros((nf + N, nf + N))
    K[:nf, :nf] = Mm
    K[:nf, nf:] = -B.T
    K[nf:, :nf] = B
    rhs = np.concatenate([rhs_u, rhs_p])
    for fi, z in fixed.items():
        K[fi, :] = 0.0
        K[fi, fi] = 1.0
        rhs[fi] = z
    sol = np.linalg.solve(K, rhs)
    return sol[nf:], sol[:nf], faces
