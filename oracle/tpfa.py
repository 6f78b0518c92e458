"""Two-point-flux systems on boxes of Cartesian cells (oracle, test-only).

Section 2 (paragraph after the local problems eq111dtilde/eq122dtilde) states
that lowest-order Raviart-Thomas spaces on uniform Cartesian cells, with
midpoint/trapezoid quadrature, reduce to a cell-centred finite-difference
system in the pressure alone.  Written out for cell size ``h`` in ``d``
dimensions (face area ``|e| = h^(d-1)``, cell volume ``h^d``):

* half transmissibility of cell c towards a face: ``2 K_c |e| / h``;
* interior face between c and c': ``T_e = |e| K_H / h`` with ``K_H`` the
  harmonic mean of ``K_c`` and ``K_c'``; the outward normal velocity from c is
  ``u_e = T_e (p_c - p_c') / |e|``;
* a diagonal permeability tensor (Section 2 allows any symmetric positive
  definite K) enters a face normal to axis a only through its a-th diagonal
  entry: every ``K_c`` above is then ``K_c^(a)`` of the face's axis, the
  two-point flux being consistent for a diagonal tensor on a Cartesian grid;
* Robin face (``-beta u.n + p = lam``, equation genRobin): the face pressure is
  ``pi = lam + beta u``, and with the half-cell relation
  ``u = 2 K_c (p_c - pi) / h`` one gets ``|e| u = T^R (p_c - lam)`` with
  ``T^R = |e| / (h / (2 K_c) + beta)``;
* Dirichlet face (pressure g): ``|e| u = 2 K_c |e| / h (p_c - g)``;
* Neumann face (normal velocity z, equation eq1d): ``|e| u = |e| z``.

Mass balance in every cell (equation eq1b integrated over the cell) gives the
symmetric positive (semi)definite system ``A p = b`` with
``b_c = f_c h^d + sum_Rob T^R lam + sum_Dir T^D g - sum_Neu |e| z``.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class Grid:
    """Uniform Cartesian grid; cell arrays are flat in x-fastest order."""

    def __init__(self, ncell, h, perm):
        """perm: K per cell (scalar K), or shape (d, cells) / (d, *cells) for
        a diagonal tensor: row a holds the entry of axis a."""
        self.n = tuple(int(v) for v in ncell)
        self.d = len(self.n)
        self.h = float(h)
        N = int(np.prod(self.n))
        k = np.asarray(perm, dtype=np.float64)
        if k.size == N:
            self.Ka = np.tile(k.ravel(), (self.d, 1))
            self.isotropic = True
        else:
            assert k.size == self.d * N
            self.Ka = np.ascontiguousarray(k.reshape(self.d, N))
            self.isotropic = False
        self.stride = tuple(int(np.prod(self.n[:a])) for a in range(self.d))
        self.area = self.h ** (self.d - 1)
        self.vol = self.h ** self.d

    @property
    def ncells(self):
        return int(np.prod(self.n))

    def flat(self, coords):
        coords = np.asarray(coords)
        return sum(coords[..., a] * self.stride[a] for a in range(self.d))

    def coords(self, flat):
        flat = np.asarray(flat)
        out = []
        for a in range(self.d):
            out.append((flat // self.stride[a]) % self.n[a])
        return np.stack(out, axis=-1)

    def k(self, c, a):
        """K of cells c in the direction of axis a."""
        return self.Ka[a][c]

    def k_harmonic(self, c, c2, a):
        k1 = self.Ka[a][c]
        k2 = self.Ka[a][c2]
        return 2.0 * k1 * k2 / (k1 + k2)

    def trans(self, c, c2, a):
        """Transmissibility |e| K_H / h of the faces normal to axis a between
        cells c and c2."""
        return self.area * self.k_harmonic(c, c2, a) / self.h

    def half_trans(self, c, a):
        return 2.0 * self.Ka[a][c] * self.area / self.h


def box_coords(lo, hi):
    """Global coordinates of the cells of box [lo, hi) in x-fastest order."""
    d = len(lo)
    axes = [np.arange(lo[a], hi[a]) for a in range(d)]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")
    return np.stack([m.ravel() for m in mesh[::-1]], axis=-1)


def side_local(lo, hi, side):
    """Local indices (in box order) of the box cells adjacent to one side.

    ``side = 2a + s`` (s = 0 low, 1 high).  The cells come out in x-fastest
    order over the remaining axes, which is also the order of the side's faces.
    """
    m = [hi[a] - lo[a] for a in range(len(lo))]
    a, s = divmod(side, 2)
    loc = box_coords([0] * len(lo), m)
    sel = loc[:, a] == (0 if s == 0 else m[a] - 1)
    return np.nonzero(sel)[0]


def boundary_face_index(grid, coords, side):
    """Index of the face of global side ``side`` that a boundary cell touches."""
    a = side // 2
    idx = np.zeros(coords.shape[0], dtype=np.int64)
    mult = 1
    for b in range(grid.d):
        if b == a:
            continue
        idx += coords[:, b] * mult
        mult *= grid.n[b]
    return idx


class BoxProblem:
    """TPFA matrix of one box with its boundary-face bookkeeping.

    Box sides lying on the domain boundary take the global condition of that
    side (``bc_type[side]`` in {"D", "N"}); every other box side is a Robin
    side whose parameter per face comes from ``beta_fn(axis, inner, outer)``
    (global flat cell indices on both sides of the face).
    """

    def __init__(self, grid, bc_type, lo, hi, beta_fn):
        self.grid = grid
        self.lo = tuple(int(v) for v in lo)
        self.hi = tuple(int(v) for v in hi)
        d = grid.d
        self.coords = box_coords(self.lo, self.hi)
        self.gidx = grid.flat(self.coords)
        nloc = self.gidx.size
        self.nloc = nloc
        local_of = {int(g): k for k, g in enumerate(self.gidx)}
        self.local_of = local_of
        rows, cols, vals = [], [], []
        diag = np.zeros(nloc)
        m = [self.hi[a] - self.lo[a] for a in range(d)]
        self.robin = {}   # side -> dict(local, outer, beta, TR)
        self.bcf = {}     # side -> dict(local, face, type, coef)
        loc = box_coords([0] * d, m)
        for a in range(d):
            # interior faces inside the box along axis a
            sel = np.nonzero(loc[:, a] < m[a] - 1)[0]
            nb = sel + int(np.prod(m[:a]))
            T = grid.trans(self.gidx[sel], self.gidx[nb], a)
            rows += [sel, nb]
            cols += [nb, sel]
            vals += [-T, -T]
            np.add.at(diag, sel, T)
            np.add.at(diag, nb, T)
            for s in (0, 1):
                side = 2 * a + s
                lc = side_local(self.lo, self.hi, side)
                gc = self.gidx[lc]
                on_boundary = (s == 0 and self.lo[a] == 0) or (s == 1 and self.hi[a] == grid.n[a])
                if on_boundary:
                    typ = bc_type[side]
                    coef = grid.half_trans(gc, a) if typ == "D" else np.zeros(lc.size)
                    if typ == "D":
                        np.add.at(diag, lc, coef)
                    self.bcf[side] = dict(local=lc, face=boundary_face_index(grid, self.coords[lc], side),
                                          type=typ, coef=coef)
                else:
                    oc = self.coords[lc].copy()
                    oc[:, a] += -1 if s == 0 else 1
                    og = grid.flat(oc)
                    beta = np.asarray(beta_fn(a, gc, og), dtype=np.float64) * np.ones(lc.size)
                    TR = grid.area / (grid.h / (2.0 * grid.k(gc, a)) + beta)
                    np.add.at(diag, lc, TR)
                    self.robin[side] = dict(local=lc, outer=og, beta=beta, TR=TR)
        rows.append(np.arange(nloc))
        cols.append(np.arange(nloc))
        vals.append(diag)
        self.A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(nloc, nloc))
        self._lu = None

    @property
    def robin_sides(self):
        return sorted(self.robin.keys())

    def rhs(self, f=None, bc_value=None, lam=None):
        """Right-hand side for source density ``f`` (global array or None),
        boundary data ``bc_value`` (list per side, or None for zero) and Robin
        data ``lam`` (dict side -> per-face array, missing sides are zero)."""
        g = self.grid
        b = np.zeros(self.nloc)
        if f is not None:
            b += np.asarray(f).ravel()[self.gidx] * g.vol
        if bc_value is not None:
            for side, e in self.bcf.items():
                val = np.asarray(bc_value[side])[e["face"]]
                if e["type"] == "D":
                    np.add.at(b, e["local"], e["coef"] * val)
                else:
                    np.add.at(b, e["local"], -g.area * val)
        if lam is not None:
            for side, vec in lam.items():
                e = self.robin[side]
                np.add.at(b, e["local"], e["TR"] * np.asarray(vec))
        return b

    def solve(self, b):
        if self._lu is None:
            self._lu = spla.splu(self.A.tocsc())
        return self._lu.solve(np.asarray(b, dtype=np.float64))

    def robin_velocity(self, p, side, lam):
        """Outward normal velocity on a Robin side for box solution p."""
        e = self.robin[side]
        return e["TR"] * (p[e["local"]] - lam) / self.grid.area


def is_pure_neumann(bc_type):
    return all(t == "N" for t in bc_type)


def fine_solve(grid, bc_type, bc_value, f):
    """Solve the non-decomposed fine problem (equations eqglo1-eqglo2).

    With no pressure boundary the system is singular (constant null vector);
    the first cell's equation is replaced by p_0 = 0 (it is redundant because
    the data are compatible) and the result is shifted to zero mean.
    """
    box = BoxProblem(grid, bc_type, [0] * grid.d, grid.n, lambda a, c, o: 0.0)
    b = box.rhs(f=f, bc_value=bc_value)
    A = box.A
    if is_pure_neumann(bc_type):
        A = A.tolil()
        A[0, :] = 0.0
        A[0, 0] = 1.0
        A = A.tocsr()
        b = b.copy()
        b[0] = 0.0
        p = spla.spsolve(A.tocsc(), b)
        p = p - p.mean()
    else:
        p = box.solve(b)
    out = np.empty(grid.ncells)
    out[box.gidx] = p
    return out


def cell_face_velocity(grid, p, bc_type, bc_value, face_override=None):
    """Outward normal velocity on every face of every cell, shape (N, 2d).

    Interior faces use the two-point flux of ``p``; domain-boundary faces use
    the boundary condition.  ``face_override(cells, side)`` may return an
    array (NaN where not overridden) to replace interior-face values, which is
    how subdomain-owned interface fluxes are inserted.
    """
    d = grid.d
    N = grid.ncells
    allc = np.arange(N)
    co = grid.coords(allc)
    out = np.zeros((N, 2 * d))
    for a in range(d):
        for s in (0, 1):
            side = 2 * a + s
            nbc = co.copy()
            nbc[:, a] += -1 if s == 0 else 1
            inside = (nbc[:, a] >= 0) & (nbc[:, a] < grid.n[a])
            cin = allc[inside]
            cn = grid.flat(nbc[inside])
            out[cin, side] = grid.trans(cin, cn, a) * (p[cin] - p[cn]) / grid.area
            cb = allc[~inside]
            face = boundary_face_index(grid, co[cb], side)
            val = np.asarray(bc_value[side])[face]
            if bc_type[side] == "D":
                out[cb, side] = grid.half_trans(cb, a) * (p[cb] - val) / grid.area
            else:
                out[cb, side] = val
            if face_override is not None:
                ov = face_override(cin, side)
                if ov is not None:
                    m = ~np.isnan(ov)
                    out[cin[m], side] = ov[m]
    return out
