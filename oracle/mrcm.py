"""MRCM-O and MRCM-OS, step by step (oracle, test-only).

Follows Algorithm 1 (computational strategy) of the paper:

Step 1-2  informed spaces: N local Darcy problems per oversampled box with
          seed Robin data (the oversampling problem), whose velocity and
          pressure traces on Gamma_i give phi_i^k (equation informed_space);
          the solutions restricted to Omega_i are the multiscale basis
          functions (Remark after equation int_pjump).
Step 3-4  particular problem on Omega_i with zero Robin data (equations
          eq111dbar-eq122dbar) and the interface system (equations int_ujump,
          int_pjump) tested with the bases of M_H and V_H.
Step 5    interface solve and MRCM-O solution (equations eq:addu, eq:addp,
          eq:uhatphat).
Step 6-7  smoothing steps (Section 3): colored Robin re-solves on the
          oversampled boxes, with Robin data taken from the current solution.

Conventions (the readings of silent or ambiguous passages):

* Subdomains are boxes of ``sub`` cells per axis, numbered lexicographically
  with axis 0 fastest.  The oversampled box grows each side by ``overlap``
  cells and is clipped to the domain.  Sides are ``2a + s`` (s = 0 low, 1 high).
* beta per face is ``alpha H_a / K_H`` (equation for beta after genRobin) with
  ``H_a = sub[a] h`` and ``K_H`` the harmonic mean across that face; or a
  constant in ``beta_mode == "const"``.
* Seeds on each Robin side of the oversampled box: ``const`` -> {1};
  ``linear`` -> {1, t_b} with t_b in (-1, 1) along each tangential axis of that
  side; ``fine`` -> indicators of the faces of that side whose tangential
  position lies inside Omega_i (the count needed by Proposition 2's remark).
  The same families (measured on the coarse interface) are the M_H / V_H bases.
* The pressure trace on a face is the half-cell value
  ``pi = p_c - u h / (2 K_c)`` from the inside cell.
* The unique normal on Gamma_ij points out of the lower-indexed subdomain, so
  pressure rows carry +1 for the lower index and -1 for the higher one.
* With no pressure boundary the interface system has the constant mode
  (all constant seeds = 1) in its kernel; the first constant flux row is
  replaced by the gauge ``X_0^0 = 0`` and the final pressure is shifted to
  zero mean.
* Smoothing colors are the 2^d parities of the subdomain index, processed in
  increasing order; all boxes of one color read the state as it was at the
  start of that color and are then written together.  With ``overlap == 0``
  the Robin data of a face come from the neighbour's own flux and trace.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .tpfa import Grid, BoxProblem, box_coords, side_local, is_pure_neumann, \
    cell_face_velocity, fine_solve


class Partition:
    def __init__(self, ncell, sub, overlap):
        self.n = tuple(int(v) for v in ncell)
        self.d = len(self.n)
        self.S = tuple(int(v) for v in sub)
        self.l = int(overlap)
        for a in range(self.d):
            if self.n[a] % self.S[a]:
                raise ValueError("cells per axis must be a multiple of the subdomain size")
            if not (0 <= self.l <= self.S[a] - 1):
                raise ValueError("overlap must satisfy 0 <= l <= S - 1")
        self.M = tuple(self.n[a] // self.S[a] for a in range(self.d))
        self.nsub = int(np.prod(self.M))
        self.sstride = tuple(int(np.prod(self.M[:a])) for a in range(self.d))

    def sub_coords(self, i):
        return tuple((i // self.sstride[a]) % self.M[a] for a in range(self.d))

    def omega(self, i):
        ic = self.sub_coords(i)
        lo = tuple(ic[a] * self.S[a] for a in range(self.d))
        hi = tuple(lo[a] + self.S[a] for a in range(self.d))
        return lo, hi

    def omega_hat(self, i):
        lo, hi = self.omega(i)
        lo2 = tuple(max(lo[a] - self.l, 0) for a in range(self.d))
        hi2 = tuple(min(hi[a] + self.l, self.n[a]) for a in range(self.d))
        return lo2, hi2

    def neighbor(self, i, side):
        a, s = divmod(side, 2)
        ic = self.sub_coords(i)
        t = ic[a] + (1 if s else -1)
        if t < 0 or t >= self.M[a]:
            return None
        return i + (1 if s else -1) * self.sstride[a]

    def gamma_sides(self, i):
        return [q for q in range(2 * self.d) if self.neighbor(i, q) is not None]

    def color(self, i):
        ic = self.sub_coords(i)
        return sum((ic[a] % 2) << a for a in range(self.d))

    def interfaces(self):
        """(i, axis, j) with i < j, ordered by i then axis."""
        out = []
        for i in range(self.nsub):
            for a in range(self.d):
                j = self.neighbor(i, 2 * a + 1)
                if j is not None:
                    out.append((i, a, j))
        return out

    def owner(self, grid_coords):
        return sum((grid_coords[..., a] // self.S[a]) * self.sstride[a] for a in range(self.d))


def make_beta(grid, part, mode, value):
    if mode == "const":
        return lambda a, c, o: np.full(np.size(c), float(value))
    if mode == "alpha":
        return lambda a, c, o: float(value) * part.S[a] * grid.h / grid.k_harmonic(c, o, a)
    raise ValueError(mode)


def _tangential(lo, hi, side, d):
    """Face-centre coordinates t_b in (-1, 1) of a side of box [lo, hi)."""
    a = side // 2
    m = [hi[b] - lo[b] for b in range(d)]
    loc = box_coords([0] * d, m)
    lc = side_local(lo, hi, side)
    ts = []
    for b in range(d):
        if b == a:
            continue
        ts.append((2.0 * loc[lc, b] + 1.0) / m[b] - 1.0)
    return ts, loc[lc]


def side_family(space, lo, hi, side, d, window=None):
    """Basis vectors over the faces of one side of box [lo, hi).

    ``window`` (global lo/hi of Omega_i) selects the faces used by the
    ``fine`` family.  Returns a list of per-face arrays; the first vector of
    the ``const`` and ``linear`` families is the constant one.
    """
    ts, loc = _tangential(lo, hi, side, d)
    nf = loc.shape[0]
    if space == "const":
        return [np.ones(nf)]
    if space == "linear":
        return [np.ones(nf)] + [t.copy() for t in ts]
    if space == "fine":
        a = side // 2
        glob = loc + np.asarray(lo)
        keep = np.ones(nf, dtype=bool)
        for b in range(d):
            if b == a:
                continue
            keep &= (glob[:, b] >= window[0][b]) & (glob[:, b] < window[1][b])
        vecs = []
        for k in np.nonzero(keep)[0]:
            v = np.zeros(nf)
            v[k] = 1.0
            vecs.append(v)
        return vecs
    raise ValueError(space)


class MRCM:
    """One MRCM-OS solve of the fine problem described by a workload record."""

    def __init__(self, wl):
        self.wl = wl
        self.grid = Grid(wl.ncell, wl.h, wl.perm)
        self.part = Partition(wl.ncell, wl.sub, wl.overlap)
        self.bc_type = tuple(wl.bc_type)
        self.bc_value = [np.asarray(v, dtype=np.float64) for v in wl.bc_value]
        self.f = np.asarray(wl.source, dtype=np.float64).ravel()
        self.space = wl.space
        self.beta_mbf = make_beta(self.grid, self.part, wl.beta_mode, wl.beta_mbf)
        self.beta_sm = make_beta(self.grid, self.part, wl.beta_mode, wl.beta_smooth)
        self.same_beta = (wl.beta_mbf == wl.beta_smooth)
        self.neumann = is_pure_neumann(self.bc_type)
        self.counts = dict(factor=0, solves=0)

    # ------------------------------------------------------------------ Step 1-2
    def _gamma_traces(self, box, i, P, lam, beta_fn):
        """u, pi, phi on every Gamma_i side of subdomain i for box solution P.

        u is the outward (from Omega_i) normal velocity; pi the half-cell
        pressure trace from the inside cell; phi = -beta u + pi
        (equation informed_space)."""
        g = self.grid
        lo, hi = self.part.omega(i)
        out = {}
        for side in self.part.gamma_sides(i):
            a, s = divmod(side, 2)
            co = box_coords(lo, hi)[side_local(lo, hi, side)]
            c = g.flat(co)
            oc = co.copy()
            oc[:, a] += -1 if s == 0 else 1
            c2 = g.flat(oc)
            inner = np.array([box.local_of[int(v)] for v in c])
            if all(int(v) in box.local_of for v in c2):
                outer = np.array([box.local_of[int(v)] for v in c2])
                u = g.trans(c, c2, a) * (P[inner] - P[outer]) / g.area
            else:
                # no oversampling: Gamma_i is the Robin side of the box itself
                u = box.robin_velocity(P, side, lam.get(side, 0.0))
            pi = P[inner] - u * g.h / (2.0 * g.k(c, a))
            beta = beta_fn(a, c, c2) * np.ones(c.size)
            out[side] = dict(u=u, pi=pi, phi=-beta * u + pi, beta=beta)
        return out

    def build_basis(self):
        part, g = self.part, self.grid
        self.boxes = []
        self.mbf = []
        for i in range(part.nsub):
            lo, hi = part.omega_hat(i)
            box = BoxProblem(g, self.bc_type, lo, hi, self.beta_mbf)
            self.counts["factor"] += 1
            wlo, whi = part.omega(i)
            seeds = []
            for side in box.robin_sides:
                for vec in side_family(self.space, lo, hi, side, g.d, window=(wlo, whi)):
                    seeds.append((side, vec))
            om = box_coords(wlo, whi)
            om_loc = np.array([box.local_of[int(v)] for v in g.flat(om)])
            rec = dict(seeds=seeds, P=[], traces=[])
            for side, vec in seeds:
                lam = {side: vec}
                P = box.solve(box.rhs(lam=lam))
                self.counts["solves"] += 1
                rec["P"].append(P[om_loc])
                rec["traces"].append(self._gamma_traces(box, i, P, lam, self.beta_mbf))
            self.boxes.append(box)
            self.mbf.append(rec)
        self.nseed = [len(r["seeds"]) for r in self.mbf]
        self.offset = np.concatenate([[0], np.cumsum(self.nseed)]).astype(int)

    # ------------------------------------------------------------------ Step 4
    def particular(self):
        part, g = self.part, self.grid
        self.part_sol = []
        for i in range(part.nsub):
            lo, hi = part.omega(i)
            box = BoxProblem(g, self.bc_type, lo, hi, self.beta_mbf)
            self.counts["factor"] += 1
            pbar = box.solve(box.rhs(f=self.f, bc_value=self.bc_value))
            self.counts["solves"] += 1
            tr = {}
            for side in part.gamma_sides(i):
                u = box.robin_velocity(pbar, side, 0.0)
                beta = box.robin[side]["beta"]
                tr[side] = dict(u=u, pi=beta * u)
            self.part_sol.append(dict(p=pbar, traces=tr))

    # ------------------------------------------------------------------ Step 3-5
    def interface_family(self, i, side):
        lo, hi = self.part.omega(i)
        return side_family(self.space, lo, hi, side, self.grid.d, window=(lo, hi))

    def assemble_interface(self):
        part, g = self.part, self.grid
        nX = int(self.offset[-1])
        rows, cols, vals, rhs = [], [], [], []
        r = 0
        self.row_info = []
        for (i, a, j) in part.interfaces():
            qi, qj = 2 * a + 1, 2 * a
            fam = self.interface_family(i, qi)
            for kind in ("flux", "pressure"):
                sign_j = 1.0 if kind == "flux" else -1.0
                for mu in fam:
                    w = g.area * mu
                    acc = 0.0
                    for sub, q, sg in ((i, qi, 1.0), (j, qj, sign_j)):
                        for k in range(self.nseed[sub]):
                            t = self.mbf[sub]["traces"][k][q]
                            coef = t["u"] if kind == "flux" else t["beta"] * t["u"] + t["phi"]
                            rows.append(r)
                            cols.append(self.offset[sub] + k)
                            vals.append(sg * np.dot(w, coef))
                        pt = self.part_sol[sub]["traces"][q]
                        acc += sg * np.dot(w, pt["u"] if kind == "flux" else pt["pi"])
                    rhs.append(-acc)
                    self.row_info.append((i, a, j, kind))
                    r += 1
        G = sp.csr_matrix((vals, (rows, cols)), shape=(r, nX))
        rhs = np.asarray(rhs)
        if r != nX:
            raise ValueError("interface system is not square (Proposition 1 violated): %d x %d" % (r, nX))
        if self.neumann:
            G = G.tolil()
            G[0, :] = 0.0
            G[0, 0] = 1.0
            G = G.tocsr()
            rhs[0] = 0.0
        self.G = G
        self.r = rhs
        return G, rhs

    def solve_interface(self):
        self.X = spla.spsolve(self.G.tocsc(), self.r)
        self.combine()

    def combine(self):
        """MRCM-O solution: p = pbar + sum_k X_k P_k, Gamma fluxes likewise."""
        part, g = self.part, self.grid
        p = np.zeros(g.ncells)
        self.gflux = []
        for i in range(part.nsub):
            lo, hi = part.omega(i)
            Xi = self.X[self.offset[i]:self.offset[i + 1]]
            pi = self.part_sol[i]["p"].copy()
            for k in range(self.nseed[i]):
                pi += Xi[k] * self.mbf[i]["P"][k]
            p[g.flat(box_coords(lo, hi))] = pi
            fl = {}
            for side in part.gamma_sides(i):
                u = self.part_sol[i]["traces"][side]["u"].copy()
                for k in range(self.nseed[i]):
                    u += Xi[k] * self.mbf[i]["traces"][k][side]["u"]
                fl[side] = u
            self.gflux.append(fl)
        self.p = p

    # ------------------------------------------------------------------ Step 6-7
    def _smooth_boxes(self):
        if self.same_beta:
            return self.boxes
        if not hasattr(self, "_sboxes"):
            self._sboxes = []
            for i in range(self.part.nsub):
                lo, hi = self.part.omega_hat(i)
                self._sboxes.append(BoxProblem(self.grid, self.bc_type, lo, hi, self.beta_sm))
                self.counts["factor"] += 1
        return self._sboxes

    def _robin_data(self, box, i):
        """lambda = -beta u.n + pi on every Robin side of box i (Section 3,
        item 3), from the current state."""
        g, part = self.grid, self.part
        lam = {}
        for side in box.robin_sides:
            e = box.robin[side]
            a = side // 2
            c = box.gidx[e["local"]]
            o = e["outer"]
            if part.l > 0:
                u = g.trans(c, o, a) * (self.p[c] - self.p[o]) / g.area
                pi = self.p[c] - u * g.h / (2.0 * g.k(c, a))
            else:
                j = part.neighbor(i, side)
                uj = self.gflux[j][side ^ 1]           # neighbour's outward flux
                pij = self.p[o] - uj * g.h / (2.0 * g.k(o, a))
                u = -uj
                pi = pij
            lam[side] = -e["beta"] * u + pi
        return lam

    def smooth(self, nsteps):
        part, g = self.part, self.grid
        boxes = self._smooth_boxes()
        for _ in range(nsteps):
            for color in range(2 ** g.d):
                members = [i for i in range(part.nsub) if part.color(i) == color]
                lams = {i: self._robin_data(boxes[i], i) for i in members}
                results = {}
                for i in members:
                    box = boxes[i]
                    ph = box.solve(box.rhs(f=self.f, bc_value=self.bc_value, lam=lams[i]))
                    self.counts["solves"] += 1
                    tr = self._gamma_traces(box, i, ph, lams[i], self.beta_sm)
                    results[i] = (ph, tr)
                for i in members:
                    ph, tr = results[i]
                    box = boxes[i]
                    lo, hi = part.omega(i)
                    om = g.flat(box_coords(lo, hi))
                    self.p[om] = ph[[box.local_of[int(v)] for v in om]]
                    for side in part.gamma_sides(i):
                        self.gflux[i][side] = tr[side]["u"]

    # ------------------------------------------------------------------ outputs
    def pressure(self):
        p = self.p.copy()
        if self.neumann:
            p -= p.mean()
        return p

    def flux(self):
        """Outward velocity per cell face (N, 2d); faces on Gamma carry the
        value of the subdomain that owns the cell."""
        g, part = self.grid, self.part

        def override(cells, side):
            co = g.coords(cells)
            a, s = divmod(side, 2)
            nb = co.copy()
            nb[:, a] += -1 if s == 0 else 1
            own = part.owner(co)
            own2 = part.owner(nb)
            out = np.full(cells.size, np.nan)
            for k in np.nonzero(own != own2)[0]:
                i = int(own[k])
                lo, _ = part.omega(i)
                pos, mult = 0, 1
                for b in range(g.d):
                    if b != a:
                        pos += (int(co[k, b]) - lo[b]) * mult
                        mult *= part.S[b]
                out[k] = self.gflux[i][side][pos]
            return out

        return cell_face_velocity(g, self.p, self.bc_type, self.bc_value, face_override=override)

    def run(self, nsmooth=None):
        self.build_basis()
        self.particular()
        self.assemble_interface()
        self.solve_interface()
        self.p_mrcm_o = self.pressure()
        self.smooth(self.wl.nsmooth if nsmooth is None else nsmooth)
        return self


def solve(wl, nsmooth=None):
    """Full MRCM-OS solve; returns the solver object (pressure(), flux())."""
    return MRCM(wl).run(nsmooth)


def fine(wl):
    """Fine-grid reference solution and its face velocities."""
    g = Grid(wl.ncell, wl.h, wl.perm)
    p = fine_solve(g, wl.bc_type, wl.bc_value, wl.source)
    return p, cell_face_velocity(g, p, wl.bc_type, wl.bc_value)


def rel_l2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
