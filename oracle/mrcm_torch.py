"""MRCM-OS as a differentiable function of log K (oracle, test-only).

A second, independent CPU implementation of the same method as
``oracle/mrcm.py``, written with dense PyTorch float64 tensors so that
reverse-mode automatic differentiation yields the exact gradient of the
discrete MRCM-OS map  log K -> (pressure, face velocities).  It serves as
the FP64 CPU adjoint that the device adjoint is compared with.  Only the
geometry helpers (partition, box cell lists, seed / test-function families)
are shared with the numpy oracle; every K-dependent quantity is recomputed
here.

Steps, in the order of Algorithm 1 (Section 4):

* local TPFA systems (Section 2, the remark after the local problems): interior
  faces |e| K_H / h, Robin faces |e| / (h / (2 K_c) + beta), Dirichlet faces
  2 K_c |e| / h; beta = alpha H / K_H or a constant (equation after genRobin);
* seed solves on the oversampled boxes and their traces on Gamma_i
  (equation informed_space): u, pi = p_c - u h / (2 K_c), phi = -beta u + pi;
* particular solves on Omega_i with zero Robin data (eq111dbar - eq122dbar);
* moment equations (int_ujump, int_pjump), with the gauge row X_0 = 0 when no
  side carries a pressure condition;
* MRCM-O assembly (addu, addp, uhatphat) and the coloured smoothing steps of
  Section 3 (the neighbour's flux and trace when the boxes do not overlap);
* outputs: pressure (zero mean for the pure-Neumann problem) and the outward
  velocity on every cell face, Gamma faces carrying the owner's value.

Every linear system is solved densely with torch.linalg.solve (slow; small
cases only).
"""
import numpy as np
import torch

from .mrcm import Partition, side_family
from .tpfa import box_coords, side_local, is_pure_neumann

DT = torch.float64


class TorchMRCM:
    def __init__(self, wl, logk):
        self.wl = wl
        self.n = tuple(int(v) for v in wl.ncell)
        self.d = len(self.n)
        self.h = float(wl.h)
        self.area = self.h ** (self.d - 1)
        self.vol = self.h ** self.d
        self.N = int(np.prod(self.n))
        self.stride = tuple(int(np.prod(self.n[:a])) for a in range(self.d))
        self.K = torch.exp(logk.reshape(-1))
        self.part = Partition(wl.ncell, wl.sub, wl.overlap)
        self.bc_type = tuple(wl.bc_type)
        self.bc_value = [torch.as_tensor(np.asarray(v, dtype=np.float64)) for v in wl.bc_value]
        self.f = torch.as_tensor(np.asarray(wl.source, dtype=np.float64).ravel())
        self.space = wl.space
        self.beta_mode = wl.beta_mode
        self.neumann = is_pure_neumann(self.bc_type)

    # ------------------------------------------------------------- geometry
    def flat(self, co):
        co = np.asarray(co)
        return sum(co[..., a] * self.stride[a] for a in range(self.d))

    def kh(self, c, o):
        return 2.0 * self.K[c] * self.K[o] / (self.K[c] + self.K[o])

    def beta(self, value, a, c, o):
        if self.beta_mode == "const":
            return torch.full((len(c),), float(value), dtype=DT)
        return float(value) * self.part.S[a] * self.h / self.kh(c, o)

    # ------------------------------------------------------- local systems
    def box(self, lo, hi, bval):
        d = self.d
        co = box_coords(lo, hi)
        gidx = self.flat(co)
        n = gidx.size
        m = [hi[a] - lo[a] for a in range(d)]
        loc = box_coords([0] * d, m)
        rows, cols, vals = [], [], []
        robin, bcf = {}, {}
        for a in range(d):
            sel = np.nonzero(loc[:, a] < m[a] - 1)[0]
            nb = sel + int(np.prod(m[:a]))
            T = self.area * self.kh(gidx[sel], gidx[nb]) / self.h
            rows += [sel, nb, sel, nb]
            cols += [sel, nb, nb, sel]
            vals += [T, T, -T, -T]
            for s in (0, 1):
                side = 2 * a + s
                lc = side_local(lo, hi, side)
                gc = gidx[lc]
                if (s == 0 and lo[a] == 0) or (s == 1 and hi[a] == self.n[a]):
                    typ = self.bc_type[side]
                    coef = (2.0 * self.K[gc] * self.area / self.h if typ == "D"
                            else torch.zeros(lc.size, dtype=DT))
                    if typ == "D":
                        rows.append(lc)
                        cols.append(lc)
                        vals.append(coef)
                    face = boundary_face_index_from(self, co[lc], side)
                    bcf[side] = dict(local=lc, face=face, type=typ, coef=coef)
                else:
                    oc = co[lc].copy()
                    oc[:, a] += -1 if s == 0 else 1
                    og = self.flat(oc)
                    bt = self.beta(bval, a, gc, og)
                    TR = self.area / (self.h / (2.0 * self.K[gc]) + bt)
                    rows.append(lc)
                    cols.append(lc)
                    vals.append(TR)
                    robin[side] = dict(local=lc, outer=og, beta=bt, TR=TR)
        A = torch.zeros(n, n, dtype=DT)
        A = A.index_put((torch.as_tensor(np.concatenate(rows)), torch.as_tensor(np.concatenate(cols))),
                        torch.cat(vals), accumulate=True)
        return dict(lo=tuple(lo), hi=tuple(hi), gidx=gidx, n=n, A=A, robin=robin, bcf=bcf,
                    local_of={int(g): k for k, g in enumerate(gidx)})

    def rhs(self, B, f=False, bc=False, lam=None):
        b = torch.zeros(B["n"], dtype=DT)
        if f:
            b = b + self.f[B["gidx"]] * self.vol
        if bc:
            for side, e in B["bcf"].items():
                val = self.bc_value[side][e["face"]]
                add = e["coef"] * val if e["type"] == "D" else -self.area * val
                b = b.index_add(0, torch.as_tensor(e["local"]), add)
        if lam:
            for side, vec in lam.items():
                e = B["robin"][side]
                b = b.index_add(0, torch.as_tensor(e["local"]), e["TR"] * vec)
        return b

    def traces(self, B, i, P, lam, bval):
        """u, pi, phi, beta on every Gamma_i side for box solution P."""
        part = self.part
        lo, hi = part.omega(i)
        out = {}
        for side in part.gamma_sides(i):
            a, s = divmod(side, 2)
            co = box_coords(lo, hi)[side_local(lo, hi, side)]
            c = self.flat(co)
            oc = co.copy()
            oc[:, a] += -1 if s == 0 else 1
            c2 = self.flat(oc)
            inner = np.array([B["local_of"][int(v)] for v in c])
            if all(int(v) in B["local_of"] for v in c2):
                outer = np.array([B["local_of"][int(v)] for v in c2])
                u = self.kh(c, c2) * (P[inner] - P[outer]) / self.h
            else:
                e = B["robin"][side]
                lv = lam.get(side) if lam else None
                u = e["TR"] * (P[inner] - (lv if lv is not None else 0.0)) / self.area
            pi = P[inner] - u * self.h / (2.0 * self.K[c])
            bt = self.beta(bval, a, c, c2)
            out[side] = dict(u=u, pi=pi, phi=-bt * u + pi, beta=bt)
        return out

    # ----------------------------------------------------------- the method
    def run(self, nsmooth=None):
        wl, part = self.wl, self.part
        nsmooth = wl.nsmooth if nsmooth is None else nsmooth
        # Steps 1-2: seeds on the oversampled boxes
        self.mbf = []
        for i in range(part.nsub):
            lo, hi = part.omega_hat(i)
            B = self.box(lo, hi, wl.beta_mbf)
            wlo, whi = part.omega(i)
            seeds = []
            for side in sorted(B["robin"]):
                for vec in side_family(self.space, lo, hi, side, self.d, window=(wlo, whi)):
                    seeds.append((side, torch.as_tensor(vec)))
            om_loc = np.array([B["local_of"][int(v)] for v in self.flat(box_coords(wlo, whi))])
            rec = dict(P=[], traces=[])
            for side, vec in seeds:
                lam = {side: vec}
                P = torch.linalg.solve(B["A"], self.rhs(B, lam=lam))
                rec["P"].append(P[om_loc])
                rec["traces"].append(self.traces(B, i, P, lam, wl.beta_mbf))
            self.mbf.append(rec)
        nseed = [len(r["P"]) for r in self.mbf]
        off = np.concatenate([[0], np.cumsum(nseed)]).astype(int)
        # Step 4: particular problems on Omega_i
        self.psol = []
        for i in range(part.nsub):
            lo, hi = part.omega(i)
            B = self.box(lo, hi, wl.beta_mbf)
            pbar = torch.linalg.solve(B["A"], self.rhs(B, f=True, bc=True))
            tr = {}
            for side in part.gamma_sides(i):
                e = B["robin"][side]
                u = e["TR"] * pbar[e["local"]] / self.area
                tr[side] = dict(u=u, pi=e["beta"] * u)
            self.psol.append(dict(p=pbar, traces=tr))
        # Steps 3-5: moment equations and their solution
        nX = int(off[-1])
        G = torch.zeros(nX, nX, dtype=DT)
        r = []
        row = 0
        for (i, a, j) in part.interfaces():
            qi, qj = 2 * a + 1, 2 * a
            lo, hi = part.omega(i)
            fam = side_family(self.space, lo, hi, qi, self.d, window=(lo, hi))
            for kind in ("flux", "pressure"):
                sj = 1.0 if kind == "flux" else -1.0
                for mu in fam:
                    w = torch.as_tensor(self.area * mu)
                    acc = 0.0
                    for sub, q, sg in ((i, qi, 1.0), (j, qj, sj)):
                        for k in range(nseed[sub]):
                            t = self.mbf[sub]["traces"][k][q]
                            coef = t["u"] if kind == "flux" else t["beta"] * t["u"] + t["phi"]
                            G = G.index_put((torch.tensor([row]), torch.tensor([off[sub] + k])),
                                            (sg * torch.dot(w, coef)).reshape(1), accumulate=True)
                        pt = self.psol[sub]["traces"][q]
                        acc = acc + sg * torch.dot(w, pt["u"] if kind == "flux" else pt["pi"])
                    r.append(-acc)
                    row += 1
        r = torch.stack([torch.as_tensor(v, dtype=DT) for v in r])
        if self.neumann:
            e0 = torch.zeros(nX, dtype=DT)
            e0[0] = 1.0
            G = torch.cat([e0.reshape(1, -1), G[1:]], dim=0)
            r = torch.cat([torch.zeros(1, dtype=DT), r[1:]])
        self.X = torch.linalg.solve(G, r)
        # MRCM-O assembly
        p = torch.zeros(self.N, dtype=DT)
        self.gflux = []
        for i in range(part.nsub):
            lo, hi = part.omega(i)
            Xi = self.X[off[i]:off[i + 1]]
            pi = self.psol[i]["p"]
            for k in range(nseed[i]):
                pi = pi + Xi[k] * self.mbf[i]["P"][k]
            p = p.index_put((torch.as_tensor(self.flat(box_coords(lo, hi))),), pi)
            fl = {}
            for side in part.gamma_sides(i):
                u = self.psol[i]["traces"][side]["u"]
                for k in range(nseed[i]):
                    u = u + Xi[k] * self.mbf[i]["traces"][k][side]["u"]
                fl[side] = u
            self.gflux.append(fl)
        self.p = p
        # Steps 6-7: smoothing
        if nsmooth > 0:
            sboxes = [self.box(*part.omega_hat(i), wl.beta_smooth) for i in range(part.nsub)]
            for _ in range(nsmooth):
                for color in range(2 ** self.d):
                    members = [i for i in range(part.nsub) if part.color(i) == color]
                    res = {}
                    for i in members:
                        B = sboxes[i]
                        lam = self.robin_data(B, i)
                        ph = torch.linalg.solve(B["A"], self.rhs(B, f=True, bc=True, lam=lam))
                        res[i] = (ph, self.traces(B, i, ph, lam, wl.beta_smooth))
                    p = self.p
                    for i in members:
                        ph, tr = res[i]
                        B = sboxes[i]
                        lo, hi = part.omega(i)
                        om = self.flat(box_coords(lo, hi))
                        p = p.index_put((torch.as_tensor(om),),
                                        ph[np.array([B["local_of"][int(v)] for v in om])])
                        for side in part.gamma_sides(i):
                            self.gflux[i][side] = tr[side]["u"]
                    self.p = p
        return self

    def robin_data(self, B, i):
        part = self.part
        lam = {}
        for side in sorted(B["robin"]):
            e = B["robin"][side]
            c = B["gidx"][e["local"]]
            o = e["outer"]
            if part.l > 0:
                u = self.kh(c, o) * (self.p[c] - self.p[o]) / self.h
                pi = self.p[c] - u * self.h / (2.0 * self.K[c])
            else:
                j = part.neighbor(i, side)
                uj = self.gflux[j][side ^ 1]
                pi = self.p[o] - uj * self.h / (2.0 * self.K[o])
                u = -uj
            lam[side] = -e["beta"] * u + pi
        return lam

    # -------------------------------------------------------------- outputs
    def pressure(self):
        return self.p - self.p.mean() if self.neumann else self.p

    def flux(self):
        """Outward velocity per cell face, shape (N, 2d)."""
        d, part = self.d, self.part
        allc = np.arange(self.N)
        co = np.stack([(allc // self.stride[a]) % self.n[a] for a in range(d)], axis=-1)
        cols = []
        for a in range(d):
            for s in (0, 1):
                side = 2 * a + s
                nbc = co.copy()
                nbc[:, a] += -1 if s == 0 else 1
                inside = (nbc[:, a] >= 0) & (nbc[:, a] < self.n[a])
                cin = allc[inside]
                cn = self.flat(nbc[inside])
                col = torch.zeros(self.N, dtype=DT)
                vin = self.kh(cin, cn) * (self.p[cin] - self.p[cn]) / self.h
                # Gamma faces: the owning subdomain's flux
                own = part.owner(co[inside])
                own2 = part.owner(nbc[inside])
                gam = np.nonzero(own != own2)[0]
                if gam.size:
                    vals = []
                    for k in gam:
                        i = int(own[k])
                        lo, _ = part.omega(i)
                        pos, mult = 0, 1
                        for b in range(d):
                            if b != a:
                                pos += (int(co[cin[k], b]) - lo[b]) * mult
                                mult *= part.S[b]
                        vals.append(self.gflux[i][side][pos])
                    vin = vin.index_put((torch.as_tensor(gam),), torch.stack(vals))
                col = col.index_put((torch.as_tensor(cin),), vin)
                cb = allc[~inside]
                face = boundary_face_index_from(self, co[cb], side)
                val = self.bc_value[side][face]
                if self.bc_type[side] == "D":
                    vb = 2.0 * self.K[cb] * (self.p[cb] - val) / self.h
                else:
                    vb = val
                col = col.index_put((torch.as_tensor(cb),), vb)
                cols.append(col)
        return torch.stack(cols, dim=1)


def boundary_face_index_from(model, coords, side):
    """Face index of a domain-side face (x-fastest over the other axes)."""
    a = side // 2
    idx = np.zeros(coords.shape[0], dtype=np.int64)
    mult = 1
    for b in range(model.d):
        if b == a:
            continue
        idx += coords[:, b] * mult
        mult *= model.n[b]
    return idx


def outflow(flux, model, side=1):
    """Total outflow through one domain side: sum over its faces of |e| u.n."""
    a = side // 2
    N = model.N
    allc = np.arange(N)
    co = (allc // model.stride[a]) % model.n[a]
    cells = allc[co == (model.n[a] - 1 if side % 2 else 0)]
    return model.area * flux[torch.as_tensor(cells), side].sum()


def solve(wl, logk=None, nsmooth=None):
    """Run the method; logk defaults to the workload's field (no gradient)."""
    lk = torch.as_tensor(np.asarray(wl.logk if logk is None else logk, dtype=np.float64).ravel()) \
        if not isinstance(logk, torch.Tensor) else logk
    return TorchMRCM(wl, lk).run(nsmooth)
