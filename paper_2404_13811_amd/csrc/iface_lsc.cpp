// Two-level solver of the interface system (Algorithm 1, Step 5) for 3-D
// grids of subdomains whose layers are too large for one dense block.
//
// The unknowns and equations are split into outer layers of subdomains
// along the axis with the most subdomains (equations assigned to
// subdomains as in the cyclic reduction: the flux rows of an interface to
// its lower-indexed subdomain, the pressure rows to the higher one, each
// paired with the seeds of the same side).  Layer k's equations read
//   D_k x_k + P_L^T s_k + P_U^T t_k = r_k,
// where only the pressure rows of its lower outer interfaces (R^L_k) see
// layer k - 1, through s_k = Lr_k x_{k-1}, and only the flux rows of its
// upper outer interfaces (R^U_k) see layer k + 1, through t_k = Ur_k x_{k+1}.
//
// 1. Inner: every D_k is itself block tridiagonal over the inner layers of
//    the layer (blocks of one row of subdomains), so one batched cyclic
//    reduction of all layers at once gives Y_k = D_k^{-1} [r_k | P_L^T | P_U^T].
// 2. Reduced system over the gaps between layers: with
//    x_k = y_k - Y^L_k s_k - Y^U_k t_k,
//      s_{k+1} + Lr_{k+1} Y^L_k s_k + Lr_{k+1} Y^U_k t_k = Lr_{k+1} y_k,
//      t_k + Ur_k Y^L_{k+1} s_{k+1} + Ur_k Y^U_{k+1} t_{k+1} = Ur_k y_{k+1},
//    block tridiagonal over the gaps g = (k, k + 1) with unknowns
//    (t_k, s_{k+1}); solved by block cyclic reduction, the dense gap blocks
//    inverted by a recursive two-by-two inverse on FP64 matrix products.
// 3. Back substitution x_k = y_k - Y^L_k s_k - Y^U_k t_k.
//
// The algebra is exact (no approximation is added to the direct solve):
// the reduced system is the Schur complement of the interface system onto
// the couplings between outer layers.
//
// Columns of [r_k | P_L^T | P_U^T]: the coupling columns of each inner
// layer z side by side (its lower, then its upper couplings), the
// right-hand side last.  The unit column of a coupling row of inner layer z
// is zero outside layer z, so in the forward pass of the inner reduction a
// vector block depends only on the inner layers it has gathered: the
// block-vector products of that pass run over the column window of those
// layers (plus the right-hand side) and skip the columns that are still
// zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "mrcm_internal.h"

namespace mrcm {

namespace {

long long up32(long long v) { return (v + 31) / 32 * 32; }

// Abstract schedule of block cyclic reduction on Ml layers.  Block slots:
// D_k = k, L_k = Ml + k, U_k = 2 Ml + k, F_k = 3 Ml + k, G_k = 4 Ml + k;
// vector slots: r_k = k, g_k = Ml + k, x_k = 2 Ml + k.  A reduced L_j / U_j
// goes to the slot of the eliminated neighbour's L / U, which is no longer
// read.
struct SProd {
  int c, c0, a1, b1, a2, b2;
  double al1, al2;
};
struct SOp {
  int kind = 0;  // 0: inverses (in place; F and G slots of the block's layer
                 // are its scratch), 1: independent products and
                 // block-vector products
  std::vector<int> inv, scr;
  std::vector<SProd> prod, vec;
};

std::vector<SOp> schedule(int Ml) {
  std::vector<SOp> ops;
  std::vector<int> dsl(Ml), lsl(Ml), usl(Ml), idx(Ml);
  for (int k = 0; k < Ml; ++k) {
    dsl[k] = k;
    lsl[k] = Ml + k;
    usl[k] = 2 * Ml + k;
    idx[k] = k;
  }
  auto F = [&](int k) { return 3 * Ml + k; };
  auto G = [&](int k) { return 4 * Ml + k; };
  auto rv = [&](int k) { return k; };
  auto gv = [&](int k) { return Ml + k; };
  auto xv = [&](int k) { return 2 * Ml + k; };
  std::vector<std::vector<SProd>> back;
  while (idx.size() > 1) {
    const int L = (int)idx.size();
    SOp inv;
    inv.kind = 0;
    for (int t = 1; t < L; t += 2) {
      inv.inv.push_back(dsl[idx[t]]);
      inv.scr.push_back(F(idx[t]));
    }
    ops.push_back(inv);
    SOp a;
    a.kind = 1;
    for (int t = 1; t < L; t += 2) {
      const int k = idx[t];
      a.prod.push_back(SProd{F(k), -1, dsl[k], lsl[k], -1, -1, 1.0, 0.0});
      if (t + 1 < L) a.prod.push_back(SProd{G(k), -1, dsl[k], usl[k], -1, -1, 1.0, 0.0});
      a.vec.push_back(SProd{gv(k), -1, dsl[k], rv(k), -1, -1, 1.0, 0.0});
    }
    ops.push_back(a);
    SOp b;
    b.kind = 1;
    std::vector<int> nl(Ml, -1), nu(Ml, -1);
    for (int t = 0; t < L; t += 2) {
      const int j = idx[t];
      const bool hl = t > 0, hr = t + 1 < L;
      const int km = hl ? idx[t - 1] : -1, kp = hr ? idx[t + 1] : -1;
      SProd Dt{dsl[j], dsl[j], -1, -1, -1, -1, -1.0, -1.0};
      SProd Rt{rv(j), rv(j), -1, -1, -1, -1, -1.0, -1.0};
      if (hl) {
        Dt.a1 = lsl[j];
        Dt.b1 = G(km);
        Rt.a1 = lsl[j];
        Rt.b1 = gv(km);
      }
      if (hr) {
        (hl ? Dt.a2 : Dt.a1) = usl[j];
        (hl ? Dt.b2 : Dt.b1) = F(kp);
        (hl ? Rt.a2 : Rt.a1) = usl[j];
        (hl ? Rt.b2 : Rt.b1) = gv(kp);
      }
      if (Dt.a1 >= 0) b.prod.push_back(Dt);
      if (Rt.a1 >= 0) b.vec.push_back(Rt);
      if (hl && t - 1 > 0) {
        b.prod.push_back(SProd{lsl[km], -1, lsl[j], F(km), -1, -1, -1.0, 0.0});
        nl[j] = lsl[km];
      }
      if (hr && t + 2 < L) {
        b.prod.push_back(SProd{usl[kp], -1, usl[j], G(kp), -1, -1, -1.0, 0.0});
        nu[j] = usl[kp];
      }
    }
    ops.push_back(b);
    std::vector<SProd> bk;
    for (int t = 1; t < L; t += 2) {
      const int k = idx[t];
      SProd B{xv(k), gv(k), F(k), xv(idx[t - 1]), -1, -1, -1.0, -1.0};
      if (t + 1 < L) {
        B.a2 = G(k);
        B.b2 = xv(idx[t + 1]);
      }
      bk.push_back(B);
    }
    back.push_back(bk);
    std::vector<int> keep;
    for (int t = 0; t < L; t += 2) {
      const int j = idx[t];
      lsl[j] = nl[j];
      usl[j] = nu[j];
      keep.push_back(j);
    }
    idx.swap(keep);
  }
  const int k0 = idx[0];
  SOp last;
  last.kind = 0;
  last.inv.push_back(dsl[k0]);
  last.scr.push_back(F(k0));
  ops.push_back(last);
  SOp fin;
  fin.kind = 1;
  fin.vec.push_back(SProd{xv(k0), -1, dsl[k0], rv(k0), -1, -1, 1.0, 0.0});
  ops.push_back(fin);
  for (int lv = (int)back.size() - 1; lv >= 0; --lv) {
    SOp o;
    o.kind = 1;
    o.vec = back[lv];
    ops.push_back(o);
  }
  return ops;
}

}  // namespace

// One launch of the solver.
struct LscLaunch {
  int kind;  // 0 inverses, 1 rectangular products, 2 block-vector products (outer),
             // 3 two independent groups of products (second: off2, cnt2, shape2),
             // 4 rectangular products over their column windows (at most wmax tiles)
  int off, cnt;
  int wmax;
  int n, ld;        // inverses
  RectShape shape;  // products
  int off2, cnt2;
  RectShape shape2;
};

struct Lsc {
  // sizes
  int S = 0, Mi = 0, bpi = 0, nc = 0;  // inner systems, layers, block, right-hand sides
  int Mo = 0, ng = 0, bo = 0;          // outer layers, gaps, gap block
  int dstw = 0, wc = 0, ncol = 0;
  long long P_in = 0, R_in = 0, CV = 0, P_out = 0, V_out = 0, total = 0;
  // device
  double* buf = nullptr;
  long long* d_dst = nullptr;
  long long* d_rdst = nullptr;
  long long* d_ones = nullptr;
  long long nones = 0;
  long long* d_offs = nullptr;
  int* d_npiv = nullptr;
  BcrGemm* d_rect = nullptr;
  BcrGemv* d_gemv = nullptr;
  LscRow* d_rows = nullptr;
  long long* d_ypos = nullptr;
  int nrows = 0;
  LscCol* d_cols = nullptr;
  int ncols = 0;
  int* d_cmap = nullptr;  // per outer layer: code of every inner-solution column
  int* d_icol = nullptr;  // per outer layer: column of its j-th coupling (lower, then upper)
  int rc = 0;             // column of the right-hand side
  // launches: inner phase, outer phase
  std::vector<LscLaunch> inner, outer;
};

namespace {

// Leading part of an n x n block (n > kBcrInvMax) in the recursive
// two-by-two inverse: the largest kBcrInvMax * 2^j below n, so that the
// leading part splits into whole leaves and the recursion takes as few
// dependent launches as it can (640 = 512 + 128: five leaves of 128).
int rinv_split(int n) {
  int n1 = kBcrInvMax;
  while (2 * n1 < n) n1 *= 2;
  return n1;
}

struct Builder {
  std::vector<long long> offs;
  std::vector<int> npiv;
  std::vector<BcrGemm> rect;
  std::vector<BcrGemv> gemv;
  void inv(std::vector<LscLaunch>& L, const std::vector<long long>& blk, int n, int ld) {
    LscLaunch o{};
    o.kind = 0;
    o.off = (int)offs.size();
    o.cnt = (int)blk.size();
    o.n = n;
    o.ld = ld;
    for (long long b : blk) {
      offs.push_back(b);
      npiv.push_back(n);
    }
    L.push_back(o);
  }
  void prod(std::vector<LscLaunch>& L, const std::vector<BcrGemm>& t, const RectShape& sh) {
    if (t.empty()) return;
    LscLaunch o{};
    o.kind = 1;
    o.off = (int)rect.size();
    o.cnt = (int)t.size();
    o.shape = sh;
    rect.insert(rect.end(), t.begin(), t.end());
    L.push_back(o);
  }
  // products over column windows (wmax: most 32-column tiles of a window)
  void prodw(std::vector<LscLaunch>& L, const std::vector<BcrGemm>& t, const RectShape& sh, int wmax) {
    if (t.empty()) return;
    LscLaunch o{};
    o.kind = 4;
    o.off = (int)rect.size();
    o.cnt = (int)t.size();
    o.shape = sh;
    o.wmax = wmax;
    rect.insert(rect.end(), t.begin(), t.end());
    L.push_back(o);
  }
  void prod2(std::vector<LscLaunch>& L, const std::vector<BcrGemm>& ta, const RectShape& sa,
             const std::vector<BcrGemm>& tb, const RectShape& sb) {
    if (ta.empty() || tb.empty()) {
      prod(L, ta, sa);
      prod(L, tb, sb);
      return;
    }
    LscLaunch o{};
    o.kind = 3;
    o.off = (int)rect.size();
    o.cnt = (int)ta.size();
    o.shape = sa;
    rect.insert(rect.end(), ta.begin(), ta.end());
    o.off2 = (int)rect.size();
    o.cnt2 = (int)tb.size();
    o.shape2 = sb;
    rect.insert(rect.end(), tb.begin(), tb.end());
    L.push_back(o);
  }
  void vec(std::vector<LscLaunch>& L, const std::vector<BcrGemv>& t) {
    if (t.empty()) return;
    LscLaunch o{};
    o.kind = 2;
    o.off = (int)gemv.size();
    o.cnt = (int)t.size();
    gemv.insert(gemv.end(), t.begin(), t.end());
    L.push_back(o);
  }
  // In-place inverses of the n x n blocks at blk (leading dimension ld) by
  // the two-by-two form [A B; C D]^-1 = [A' - B' T2, B'; C', S^-1] with
  // A' = A^-1, T1 = A' B, T2 = C A', S = D - C T1, B' = -T1 S^-1,
  // C' = -S^-1 T2, recursively down to blocks of at most kBcrInvMax, which
  // one Gauss-Jordan workgroup inverts.  T1 and T2 of recursion depth d live
  // in the scratch region of each block at offset so.
  void rinv(std::vector<LscLaunch>& L, const std::vector<long long>& blk,
            const std::vector<long long>& scr, int n, int ld, long long so) {
    if (n <= kBcrInvMax) {
      inv(L, blk, n, ld);
      return;
    }
    const int n1 = rinv_split(n);
    const int n2 = n - n1;
    const long long so2 = so + 2LL * n1 * n2;
    std::vector<long long> A, B, C, D, T1, T2;
    for (size_t i = 0; i < blk.size(); ++i) {
      A.push_back(blk[i]);
      B.push_back(blk[i] + n1);
      C.push_back(blk[i] + (long long)n1 * ld);
      D.push_back(blk[i] + (long long)n1 * ld + n1);
      T1.push_back(scr[i] + so);
      T2.push_back(scr[i] + so + (long long)n1 * n2);
    }
    rinv(L, A, scr, n1, ld, so2);
    // T1 = A' B and T2 = C A' are independent: one launch
    std::vector<BcrGemm> t, u;
    for (size_t i = 0; i < blk.size(); ++i) t.push_back(BcrGemm{T1[i], -1, A[i], B[i], -1, -1, 1.0, 0.0});
    for (size_t i = 0; i < blk.size(); ++i) u.push_back(BcrGemm{T2[i], -1, C[i], A[i], -1, -1, 1.0, 0.0});
    prod2(L, t, RectShape{n1, n2, n1, ld, ld, n2}, u, RectShape{n2, n1, n1, ld, ld, n1});
    t.clear();
    for (size_t i = 0; i < blk.size(); ++i) t.push_back(BcrGemm{D[i], D[i], C[i], T1[i], -1, -1, -1.0, 0.0});
    prod(L, t, RectShape{n2, n2, n1, ld, n2, ld});
    rinv(L, D, scr, n2, ld, so2);
    // B' = -T1 S^-1 and C' = -S^-1 T2 likewise
    t.clear();
    u.clear();
    for (size_t i = 0; i < blk.size(); ++i) t.push_back(BcrGemm{B[i], -1, T1[i], D[i], -1, -1, -1.0, 0.0});
    for (size_t i = 0; i < blk.size(); ++i) u.push_back(BcrGemm{C[i], -1, D[i], T2[i], -1, -1, -1.0, 0.0});
    prod2(L, t, RectShape{n1, n2, n2, n2, ld, ld}, u, RectShape{n2, n1, n2, ld, n1, ld});
    t.clear();
    for (size_t i = 0; i < blk.size(); ++i) t.push_back(BcrGemm{A[i], A[i], B[i], T2[i], -1, -1, -1.0, 0.0});
    prod(L, t, RectShape{n1, n1, n2, ld, n1, ld});
  }
};

// Scratch doubles the recursive inverse of an n x n block needs.
long long rinv_scratch(int n) {
  if (n <= kBcrInvMax) return 0;
  const int n1 = rinv_split(n);
  const int n2 = n - n1;
  return 2LL * n1 * n2 + std::max(rinv_scratch(n1), rinv_scratch(n2));
}

template <typename T>
hipError_t upload(T*& d, const std::vector<T>& h) {
  if (h.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)&d, h.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

void lsc_destroy(Lsc* L) {
  if (!L) return;
  auto f = [](auto*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
  };
  f(L->buf); f(L->d_dst); f(L->d_rdst); f(L->d_ones); f(L->d_offs); f(L->d_npiv);
  f(L->d_rect); f(L->d_gemv); f(L->d_rows); f(L->d_ypos); f(L->d_cols); f(L->d_cmap); f(L->d_icol);
  delete L;
}

Lsc* lsc_create(const Geo& g, const std::vector<Iface>& ifc, const std::vector<int>& seed_off,
                const std::vector<int>& seeds_per_side, int nX, std::string* err,
                hipError_t* herr) {
  *herr = hipSuccess;
  auto bad = [&](const char* m) -> Lsc* {
    if (err) *err = m;
    return nullptr;
  };
  const int d = g.d;
  if (d != 3 || nX <= 0) return bad("the two-level interface solver is for 3-D grids");
  // outer axis: most subdomains; inner axis: the larger of the other two
  int ao = 0;
  for (int a = 1; a < 3; ++a)
    if (g.M[a] > g.M[ao]) ao = a;
  int ai = -1, at = -1;
  for (int a = 0; a < 3; ++a) {
    if (a == ao) continue;
    if (ai < 0 || g.M[a] > g.M[ai]) {
      at = ai;
      ai = a;
    } else {
      at = a;
    }
  }
  if (at < 0 || g.M[ao] < 2) return bad("two-level interface solver needs two outer layers");
  const int nsub = g.nsub;
  auto coord = [&](int i, int a) {
    int r = i;
    for (int b = 0; b < a; ++b) r /= g.M[b];
    return r % g.M[a];
  };
  auto nbr = [&](int i, int q) {
    const int a = q >> 1;
    const int t = coord(i, a) + ((q & 1) ? 1 : -1);
    if (t < 0 || t >= g.M[a]) return -1;
    int stride = 1;
    for (int b = 0; b < a; ++b) stride *= g.M[b];
    return i + ((q & 1) ? stride : -stride);
  };
  std::vector<int> ifc_of(3 * nsub, -1);
  for (size_t k = 0; k < ifc.size(); ++k) ifc_of[3 * ifc[k].i + ifc[k].axis] = (int)k;
  Lsc* Lp = new Lsc();
  Lsc& L = *Lp;
  L.S = L.Mo = g.M[ao];
  L.Mi = g.M[ai];
  L.ng = L.Mo - 1;
  // rows and columns: per (outer layer, inner layer), subdomains in order of
  // the third axis; each subdomain's sides in order, a side's seeds paired
  // with the equation rows it owns on that side
  std::vector<int> row_sys(nX, -1), row_z(nX, -1), row_loc(nX, -1);
  std::vector<int> col_sys(nX, -1), col_z(nX, -1), col_loc(nX, -1);
  std::vector<int> lsz((size_t)L.S * L.Mi, 0);
  std::vector<std::vector<int>> RLr(L.S), RUr(L.S);  // R^L / R^U rows per outer layer
  for (int k = 0; k < L.S; ++k)
    for (int z = 0; z < L.Mi; ++z) {
      int cnt = 0;
      for (int w = 0; w < g.M[at]; ++w) {
        int cc[3];
        cc[ao] = k;
        cc[ai] = z;
        cc[at] = w;
        const int i = cc[0] + g.M[0] * (cc[1] + g.M[1] * cc[2]);
        int s0 = seed_off[i];
        for (int q = 0; q < 2 * d; ++q) {
          const int j = nbr(i, q);
          if (j < 0) continue;
          const int a = q >> 1;
          const int f = ifc_of[3 * ((q & 1) ? i : j) + a];
          if (f < 0) {
            lsc_destroy(Lp);
            return bad("interface missing in the two-level plan");
          }
          const Iface& F = ifc[f];
          const int np = seeds_per_side[(size_t)i * 6 + q];
          if (np != F.nbasis) {
            lsc_destroy(Lp);
            return bad("seeds and test functions of a side differ in number");
          }
          const int r0 = F.row0 + ((q & 1) ? 0 : F.nbasis);
          for (int m = 0; m < np; ++m) {
            const int col = s0 + m, row = r0 + m;
            col_sys[col] = k;
            col_z[col] = z;
            col_loc[col] = cnt;
            row_sys[row] = k;
            row_z[row] = z;
            row_loc[row] = cnt;
            ++cnt;
            if (a == ao) {
              if (q & 1) RUr[k].push_back(row);
              else RLr[k].push_back(row);
            }
          }
          s0 += np;
        }
        if (s0 != seed_off[i + 1]) {
          lsc_destroy(Lp);
          return bad("seed count mismatch in the two-level plan");
        }
      }
      lsz[(size_t)k * L.Mi + z] = cnt;
    }
  for (int r = 0; r < nX; ++r)
    if (row_sys[r] < 0 || col_sys[r] < 0) {
      lsc_destroy(Lp);
      return bad("unassigned interface row or unknown");
    }
  int mx = 0, mlu = 0, mgap = 0;
  for (int v : lsz) mx = std::max(mx, v);
  for (int k = 0; k < L.S; ++k) mlu = std::max(mlu, (int)(RLr[k].size() + RUr[k].size()));
  for (int gi = 0; gi < L.ng; ++gi) mgap = std::max(mgap, (int)(RUr[gi].size() + RLr[gi + 1].size()));
  L.bpi = (int)up32(mx);
  if (L.bpi > kBcrMaxBlock) {
    lsc_destroy(Lp);
    return bad("inner layer blocks of the two-level solver exceed 256 unknowns");
  }
  L.nc = (int)up32(1 + mlu);
  L.ncol = 1 + mlu;
  // inner-solution columns per outer layer k: for every inner layer z its
  // lower then its upper coupling rows, the right-hand side last (column
  // RC); zc0 / zc1: the column range of inner layer z
  const int RC = mlu;
  std::vector<std::vector<int>> colL(L.S), colU(L.S);
  std::vector<int> zc0((size_t)L.S * L.Mi, 0), zc1((size_t)L.S * L.Mi, 0);
  std::vector<int> cmap((size_t)L.S * L.ncol, -1);
  for (int k = 0; k < L.S; ++k) {
    colL[k].assign(RLr[k].size(), -1);
    colU[k].assign(RUr[k].size(), -1);
    const int mLk = (int)RLr[k].size();
    int next = 0;
    for (int z = 0; z < L.Mi; ++z) {
      zc0[(size_t)k * L.Mi + z] = next;
      for (size_t jq = 0; jq < RLr[k].size(); ++jq)
        if (row_z[RLr[k][jq]] == z) {
          colL[k][jq] = next;
          cmap[(size_t)k * L.ncol + next] = (int)jq;
          ++next;
        }
      for (size_t jq = 0; jq < RUr[k].size(); ++jq)
        if (row_z[RUr[k][jq]] == z) {
          colU[k][jq] = next;
          cmap[(size_t)k * L.ncol + next] = mLk + (int)jq;
          ++next;
        }
      zc1[(size_t)k * L.Mi + z] = next;
    }
    cmap[(size_t)k * L.ncol + RC] = -2;
  }
  L.rc = RC;
  std::vector<int> icol((size_t)L.S * L.ncol, 0);
  for (int k = 0; k < L.S; ++k) {
    for (size_t jq = 0; jq < colL[k].size(); ++jq) icol[(size_t)k * L.ncol + jq] = colL[k][jq];
    for (size_t jq = 0; jq < colU[k].size(); ++jq)
      icol[(size_t)k * L.ncol + colL[k].size() + jq] = colU[k][jq];
  }
  L.bo = (int)up32(std::max(mgap, 32));
  const long long bsi = (long long)L.bpi * L.bpi, bso = (long long)L.bo * L.bo;
  // regions (each a multiple of 32 doubles)
  L.P_in = 0;
  L.R_in = L.P_in + (long long)L.S * 5 * L.Mi * bsi;
  // cross rows: R^L_k (k >= 1) and R^U_k (k <= Mo - 2), entries of another layer
  std::vector<int> crow(nX, -1);
  int ncross = 0;
  for (int k = 0; k < L.S; ++k) {
    for (int r : RLr[k]) crow[r] = ncross++;
    for (int r : RUr[k]) crow[r] = ncross++;
  }
  int maxrow = 0;
  for (const Iface& F : ifc) {
    const int ni = seed_off[F.i + 1] - seed_off[F.i], nj = seed_off[F.j + 1] - seed_off[F.j];
    maxrow = std::max(maxrow, ni + nj);
  }
  L.dstw = maxrow;
  L.wc = std::max(maxrow, 1);
  L.CV = L.R_in + (long long)L.S * 3 * L.Mi * L.bpi * L.nc;
  L.P_out = L.CV + up32((long long)ncross * L.wc);
  L.V_out = L.P_out + (long long)5 * L.ng * bso;
  L.total = L.V_out + up32(3LL * L.ng * L.bo);
  if (rinv_scratch(L.bo) > bso || rinv_scratch(L.bpi) > bsi) {
    lsc_destroy(Lp);
    return bad("scratch of the recursive inverse does not fit");
  }
  // destinations of the moments
  std::vector<long long> dst((size_t)nX * L.dstw, -1), rdst(nX, -1), ypos((size_t)ncross * L.wc, -1);
  std::vector<int> cfill(ncross, 0);
  auto yrow = [&](int col) { return (long long)col_z[col] * L.bpi + col_loc[col]; };
  for (const Iface& F : ifc) {
    const int ni = seed_off[F.i + 1] - seed_off[F.i], nj = seed_off[F.j + 1] - seed_off[F.j];
    for (int rr = 0; rr < 2 * F.nbasis; ++rr) {
      const int row = F.row0 + rr;
      const int k = row_sys[row], zr = row_z[row];
      rdst[row] = L.R_in + ((long long)k * 3 * L.Mi + zr) * L.bpi * L.nc + (long long)row_loc[row] * L.nc + RC;
      for (int e = 0; e < ni + nj; ++e) {
        const int col = e < ni ? seed_off[F.i] + e : seed_off[F.j] + (e - ni);
        const int kc = col_sys[col], zc = col_z[col];
        long long o;
        if (kc == k) {
          const int slot = zc == zr ? zr : (zc == zr - 1 ? L.Mi + zr : (zc == zr + 1 ? 2 * L.Mi + zr : -1));
          if (slot < 0) {
            lsc_destroy(Lp);
            return bad("inner system is not block tridiagonal");
          }
          o = L.P_in + ((long long)k * 5 * L.Mi + slot) * bsi + (long long)row_loc[row] * L.bpi + col_loc[col];
        } else {
          const int cr = crow[row];
          if (cr < 0 || (kc != k - 1 && kc != k + 1)) {
            lsc_destroy(Lp);
            return bad("outer coupling outside the neighbouring layers");
          }
          const int slot = cfill[cr]++;
          o = L.CV + (long long)cr * L.wc + slot;
          ypos[(size_t)cr * L.wc + slot] = yrow(col);
        }
        dst[(size_t)row * L.dstw + e] = o;
      }
    }
  }
  // ones: identity on the padded diagonal of the inner D blocks, unit
  // right-hand-side columns at the outer coupling rows, identity diagonal
  // of every gap block
  std::vector<long long> ones;
  for (int k = 0; k < L.S; ++k) {
    for (int z = 0; z < L.Mi; ++z)
      for (int p = lsz[(size_t)k * L.Mi + z]; p < L.bpi; ++p)
        ones.push_back(L.P_in + ((long long)k * 5 * L.Mi + z) * bsi + (long long)p * L.bpi + p);
    for (size_t jq = 0; jq < RLr[k].size(); ++jq) {
      const int r = RLr[k][jq];
      ones.push_back(L.R_in + ((long long)k * 3 * L.Mi + row_z[r]) * L.bpi * L.nc +
                     (long long)row_loc[r] * L.nc + colL[k][jq]);
    }
    for (size_t jq = 0; jq < RUr[k].size(); ++jq) {
      const int r = RUr[k][jq];
      ones.push_back(L.R_in + ((long long)k * 3 * L.Mi + row_z[r]) * L.bpi * L.nc +
                     (long long)row_loc[r] * L.nc + colU[k][jq]);
    }
  }
  for (int gi = 0; gi < L.ng; ++gi)
    for (int p = 0; p < L.bo; ++p) ones.push_back(L.P_out + (long long)gi * bso + (long long)p * L.bo + p);
  L.nones = (long long)ones.size();
  // rows of the reduced system
  const int Ml = L.ng;
  std::vector<LscRow> rows;
  auto ybase = [&](int k) { return L.R_in + ((long long)k * 3 * L.Mi + 2 * L.Mi) * L.bpi * L.nc; };
  for (int gi = 0; gi < L.ng; ++gi) {
    const int mU = (int)RUr[gi].size(), mL1 = (int)RLr[gi + 1].size();
    const int mLg = (int)RLr[gi].size(), mU1 = (int)RUr[gi + 1].size();
    // s_{g+1} + Lr_{g+1} Y^L_g s_g + Lr_{g+1} Y^U_g t_g = Lr_{g+1} y_g
    for (int q = 0; q < mL1; ++q) {
      const int r = RLr[gi + 1][q], cr = crow[r];
      const int pr = mU + q;
      LscRow R{};
      R.cval = L.CV + (long long)cr * L.wc;
      R.yidx = (long long)cr * L.wc;
      R.ybase = ybase(gi);
      R.ldy = L.nc;
      R.rhs = L.V_out + (long long)gi * L.bo + pr;
      R.cm = gi * L.ncol;
      R.ml = mLg;
      R.dst0 = gi > 0 ? L.P_out + (long long)(Ml + gi) * bso + (long long)pr * L.bo + (long long)RUr[gi - 1].size() : -1;
      R.dst1 = L.P_out + (long long)gi * bso + (long long)pr * L.bo;
      rows.push_back(R);
    }
    // t_g + Ur_g Y^L_{g+1} s_{g+1} + Ur_g Y^U_{g+1} t_{g+1} = Ur_g y_{g+1}
    for (int q = 0; q < mU; ++q) {
      const int r = RUr[gi][q], cr = crow[r];
      LscRow R{};
      R.cval = L.CV + (long long)cr * L.wc;
      R.yidx = (long long)cr * L.wc;
      R.ybase = ybase(gi + 1);
      R.ldy = L.nc;
      R.rhs = L.V_out + (long long)gi * L.bo + q;
      R.cm = (gi + 1) * L.ncol;
      R.ml = mL1;
      R.dst0 = L.P_out + (long long)gi * bso + (long long)q * L.bo + mU;
      R.dst1 = gi + 1 < L.ng ? L.P_out + (long long)(2 * Ml + gi) * bso + (long long)q * L.bo : -1;
      rows.push_back(R);
    }
  }
  L.nrows = (int)rows.size();
  // back substitution, one entry per unknown in unknown order
  std::vector<LscCol> cols(nX);
  for (int c = 0; c < nX; ++c) {
    const int k = col_sys[c];
    LscCol C{};
    C.xrow = ybase(k) + yrow(c) * L.nc;
    C.ml = (int)RLr[k].size();
    C.mu = (int)RUr[k].size();
    C.sofs = k > 0 ? L.V_out + (long long)(2 * Ml + k - 1) * L.bo + (long long)RUr[k - 1].size() : -1;
    C.tofs = k < L.Mo - 1 ? L.V_out + (long long)(2 * Ml + k) * L.bo : -1;
    C.cm = k * L.ncol;
    cols[c] = C;
  }
  L.ncols = nX;
  // inner reduction: all outer layers at once
  Builder B;
  {
    const std::vector<SOp> ops = schedule(L.Mi);
    auto pb = [&](int sys, int slot) { return L.P_in + ((long long)sys * 5 * L.Mi + slot) * bsi; };
    auto rb = [&](int sys, int slot) { return L.R_in + ((long long)sys * 3 * L.Mi + slot) * L.bpi * L.nc; };
    // inner layers gathered by each vector slot (r_k: layer k; a product's
    // output: the union over its inputs), so its window of columns
    std::vector<int> slo(3 * L.Mi, L.Mi), shi(3 * L.Mi, -1);
    for (int k = 0; k < L.Mi; ++k) slo[k] = shi[k] = k;
    for (const SOp& o : ops) {
      if (o.kind == 0) {
        std::vector<long long> blk, scr;
        for (int sys = 0; sys < L.S; ++sys)
          for (size_t q = 0; q < o.inv.size(); ++q) {
            blk.push_back(pb(sys, o.inv[q]));
            scr.push_back(pb(sys, o.scr[q]));
          }
        B.rinv(L.inner, blk, scr, L.bpi, L.bpi, 0);
        continue;
      }
      // windows of this op's vector outputs (inputs are never outputs of
      // the same op)
      std::vector<int> vlo(o.vec.size()), vhi(o.vec.size());
      for (size_t q = 0; q < o.vec.size(); ++q) {
        const SProd& t = o.vec[q];
        int lo = L.Mi, hi = -1;
        for (int in : {t.c0, t.b1, t.b2})
          if (in >= 0) {
            lo = std::min(lo, slo[in]);
            hi = std::max(hi, shi[in]);
          }
        vlo[q] = lo;
        vhi[q] = hi;
      }
      std::vector<BcrGemm> p, v;
      int wmax = 1;
      for (int sys = 0; sys < L.S; ++sys) {
        for (const SProd& t : o.prod)
          p.push_back(BcrGemm{pb(sys, t.c), t.c0 >= 0 ? pb(sys, t.c0) : -1, pb(sys, t.a1), pb(sys, t.b1),
                              t.a2 >= 0 ? pb(sys, t.a2) : -1, t.a2 >= 0 ? pb(sys, t.b2) : -1, t.al1, t.al2});
        for (size_t q = 0; q < o.vec.size(); ++q) {
          const SProd& t = o.vec[q];
          BcrGemm G{rb(sys, t.c), t.c0 >= 0 ? rb(sys, t.c0) : -1, pb(sys, t.a1), rb(sys, t.b1),
                    t.a2 >= 0 ? pb(sys, t.a2) : -1, t.a2 >= 0 ? rb(sys, t.b2) : -1, t.al1, t.al2};
          if (vhi[q] >= vlo[q] && !(vlo[q] == 0 && vhi[q] == L.Mi - 1)) {
            G.wc0 = zc0[(size_t)sys * L.Mi + vlo[q]];
            G.wc1 = zc1[(size_t)sys * L.Mi + vhi[q]];
            G.wcx = RC;
            // tiles: the window rounded out to 32 columns, and the tile of
            // the right-hand side
            const int t0 = G.wc0 / 32, t1 = (G.wc1 + 31) / 32, tx = RC / 32;
            wmax = std::max(wmax, std::max(t1 - t0, 0) + ((tx >= t0 && tx < t1) ? 0 : 1));
          } else {
            wmax = L.nc / 32;
          }
          v.push_back(G);
        }
      }
      for (size_t q = 0; q < o.vec.size(); ++q) {
        slo[o.vec[q].c] = vlo[q];
        shi[o.vec[q].c] = vhi[q];
      }
      const RectShape vs{L.bpi, L.nc, L.bpi, L.bpi, L.nc, L.nc};
      B.prod(L.inner, p, RectShape{L.bpi, L.bpi, L.bpi, L.bpi, L.bpi, L.bpi});
      if (wmax < L.nc / 32) B.prodw(L.inner, v, vs, wmax);
      else B.prod(L.inner, v, vs);
    }
  }
  // reduced system over the gaps
  {
    const std::vector<SOp> ops = schedule(L.ng);
    auto pb = [&](int slot) { return L.P_out + (long long)slot * bso; };
    for (const SOp& o : ops) {
      if (o.kind == 0) {
        std::vector<long long> blk, scr;
        for (size_t q = 0; q < o.inv.size(); ++q) {
          blk.push_back(pb(o.inv[q]));
          scr.push_back(pb(o.scr[q]));
        }
        B.rinv(L.outer, blk, scr, L.bo, L.bo, 0);
        continue;
      }
      std::vector<BcrGemm> p;
      for (const SProd& t : o.prod)
        p.push_back(BcrGemm{pb(t.c), t.c0 >= 0 ? pb(t.c0) : -1, pb(t.a1), pb(t.b1),
                            t.a2 >= 0 ? pb(t.a2) : -1, t.a2 >= 0 ? pb(t.b2) : -1, t.al1, t.al2});
      std::vector<BcrGemv> v;
      for (const SProd& t : o.vec) v.push_back(BcrGemv{t.c, t.c0, t.a1, t.b1, t.a2, t.b2, t.al1, t.al2});
      B.prod(L.outer, p, RectShape{L.bo, L.bo, L.bo, L.bo, L.bo, L.bo});
      B.vec(L.outer, v);
    }
  }
  // device memory
  hipError_t e = hipMalloc((void**)&L.buf, (size_t)L.total * sizeof(double));
  if (e == hipSuccess) e = upload(L.d_dst, dst);
  if (e == hipSuccess) e = upload(L.d_rdst, rdst);
  if (e == hipSuccess) e = upload(L.d_ones, ones);
  if (e == hipSuccess) e = upload(L.d_offs, B.offs);
  if (e == hipSuccess) e = upload(L.d_npiv, B.npiv);
  if (e == hipSuccess) e = upload(L.d_rect, B.rect);
  if (e == hipSuccess) e = upload(L.d_gemv, B.gemv);
  if (e == hipSuccess) e = upload(L.d_rows, rows);
  if (e == hipSuccess) e = upload(L.d_ypos, ypos);
  if (e == hipSuccess) e = upload(L.d_cols, cols);
  if (e == hipSuccess) e = upload(L.d_cmap, cmap);
  if (e == hipSuccess) e = upload(L.d_icol, icol);
  if (e != hipSuccess) {
    *herr = e;
    if (err) *err = hipGetErrorString(e);
    lsc_destroy(Lp);
    return nullptr;
  }
  return Lp;
}

BcrMap lsc_map(const Lsc* L) {
  BcrMap m;
  m.pool = L->buf;
  m.dst = L->d_dst;
  m.rdst = L->d_rdst;
  m.dstw = L->dstw;
  return m;
}

hipError_t lsc_prepare(Lsc* L, hipStream_t s) {
  // zeros where the moments scatter (the inner D, L, U blocks and right-hand
  // sides, the gap blocks D, L, U and right-hand sides) and in the inner g
  // vectors, which the windowed forward products write only in part; the
  // F and G blocks, the inner x vectors and the gap g and x vectors are
  // written whole before they are read (the cross values are read only
  // where the moments wrote them)
  const long long bsi = (long long)L->bpi * L->bpi, bso = (long long)L->bo * L->bo;
  const long long vsi = (long long)L->bpi * L->nc;
  const ZeroRun runs[4] = {
      {L->P_in, 3LL * L->Mi * bsi, 5LL * L->Mi * bsi, L->S},
      {L->R_in, 2LL * L->Mi * vsi, 3LL * L->Mi * vsi, L->S},
      {L->P_out, 3LL * L->ng * bso, 0, 1},
      {L->V_out, (long long)L->ng * L->bo, 0, 1},
  };
  return launch_fill_ones(L->buf, runs, 4, L->d_ones, L->nones, s);
}

namespace {
hipError_t run(Lsc* L, const std::vector<LscLaunch>& ops, int* flags, hipStream_t s) {
  for (const LscLaunch& o : ops) {
    hipError_t e = hipSuccess;
    if (o.kind == 0)
      e = launch_bcr_inv(L->buf, L->d_offs + o.off, L->d_npiv + o.off, o.cnt, o.n, o.ld, flags, s);
    else if (o.kind == 1)
      e = launch_rect_gemm(L->buf, L->d_rect + o.off, o.cnt, o.shape, s);
    else if (o.kind == 3)
      e = launch_rect_gemm2(L->buf, L->d_rect + o.off, o.cnt, o.shape, L->d_rect + o.off2, o.cnt2,
                            o.shape2, s);
    else if (o.kind == 4)
      e = launch_rect_gemm_win(L->buf, L->d_rect + o.off, o.cnt, o.shape, o.wmax, s);
    else
      e = launch_bcr_gemv(L->buf + L->P_out, L->buf + L->V_out, L->d_gemv + o.off, o.cnt, L->bo, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace

hipError_t lsc_solve(Lsc* L, double* X, int* flags, hipStream_t s) {
  hipError_t e = run(L, L->inner, flags, s);
  if (e == hipSuccess)
    e = launch_lsc_outer_rows(L->buf, L->d_rows, L->d_ypos, L->d_cmap, L->nrows, L->ncol, L->wc, s);
  if (e == hipSuccess) e = run(L, L->outer, flags, s);
  if (e == hipSuccess) e = launch_lsc_back(L->buf, L->d_cols, L->d_icol, L->ncols, L->rc, X, s);
  return e;
}

double lsc_bytes(const Lsc* L) { return (double)L->total * sizeof(double); }

void lsc_shape(const Lsc* L, int* out) {
  out[0] = L->S;
  out[1] = L->Mi;
  out[2] = L->bpi;
  out[3] = L->nc;
  out[4] = L->ng;
  out[5] = L->bo;
}

}  // namespace mrcm
