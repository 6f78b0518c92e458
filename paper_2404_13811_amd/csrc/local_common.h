// Device helpers for the local two-point-flux problems on boxes of cells.
//
// The lowest-order Raviart-Thomas discretisation with midpoint/trapezoid
// quadrature on uniform Cartesian cells reduces to a cell-centred system in
// the pressure (paper Section 2, remark after the local problems):
//   interior face   |e| u = T (p_c - p_c'),  T = |e| K_H / h, K_H harmonic mean
//   Robin face      |e| u = T^R (p_c - lam), T^R = |e| / (h / (2 K_c) + beta)
//   Dirichlet face  |e| u = 2 K_c |e| / h (p_c - g)
//   Neumann face    |e| u = |e| z
// (with a diagonal permeability tensor, K of a face normal to axis a is the
// entry of axis a) and mass balance per cell gives A p = b.  Cells of a box are numbered x
// fastest; the dense blocks of the block-tridiagonal matrix are the cells
// sharing the last-axis coordinate (lines in 2-D, planes in 3-D).
#pragma once
#include "mrcm_internal.h"

namespace mrcm {

__device__ __forceinline__ int gcell(const Geo& g, const int c[3]) {
  return c[0] + g.n[0] * (c[1] + g.n[1] * c[2]);
}

__device__ __forceinline__ double kharm(double a, double b) { return 2.0 * a * b / (a + b); }

// Robin parameter on the face between cells c (inside) and o (outside),
// normal along axis a (paper: beta = alpha H / K_H, or a constant).
__device__ __forceinline__ double robin_beta(const Geo& g, int a, double kc, double ko, double beta) {
  if (g.beta_mode == 1) return beta;
  return beta * (g.S[a] * g.h) / kharm(kc, ko);
}

__device__ __forceinline__ double robin_T(const Geo& g, double kc, double b) {
  return g.area / (g.h / (2.0 * kc) + b);
}

// Local coordinates of box cell `loc` (box order).
__device__ __forceinline__ void box_local(const Box& B, int loc, int u[3]) {
  int m0 = B.hi[0] - B.lo[0], m1 = B.hi[1] - B.lo[1];
  u[0] = loc % m0;
  int r = loc / m0;
  u[1] = r % m1;
  u[2] = r / m1;
}

// Face kinds of a box cell face.
enum { kFaceInterior = 0, kFaceRobin = 1, kFaceDir = 2, kFaceNeu = 3 };

__device__ __forceinline__ int face_kind(const Geo& g, const Box& B, const int c[3], int a, int s) {
  int t = c[a] + (s ? 1 : -1);
  if (off_domain(g, a, c[a], t)) return g.bc_type[2 * a + s] ? kFaceDir : kFaceNeu;
  if (t < B.lo[a] || t >= B.hi[a]) return kFaceRobin;
  return kFaceInterior;
}

// Element t (0..2) of a 3-array by selects, so that a runtime axis does not
// force the array into scratch memory.
__device__ __forceinline__ int pick3(const int v[3], int t) { return t == 0 ? v[0] : t == 1 ? v[1] : v[2]; }

// The tangential axes of a face normal to a (t1 unused in 2-D).
__device__ __forceinline__ void tangential(int a, int& t0, int& t1) {
  t0 = a == 0 ? 1 : 0;
  t1 = a == 2 ? 1 : 2;
}

// Index of a boundary face of domain side (a, s) touched by global cell c
// (on the y sides of a batch, member after member).
__device__ __forceinline__ int bface_index(const Geo& g, const int c[3], int a) {
  int t0, t1;
  tangential(a, t0, t1);
  const int i0 = pick3(c, t0);
  if (g.d == 3) return i0 + pick3(g.n, t0) * pick3(c, t1);
  return (a == 1 && g.cut > 0) ? i0 + g.n[0] * (c[1] / g.cut) : i0;
}

// Index of the face of side q of box [lo, hi) touched by global cell c
// (x-fastest over the tangential axes).
__device__ __forceinline__ int side_face_index(const Geo& g, const int lo[3], const int hi[3],
                                               const int c[3], int a) {
  int t0, t1;
  tangential(a, t0, t1);
  const int i0 = pick3(c, t0) - pick3(lo, t0);
  if (g.d != 3) return i0;
  return i0 + (pick3(hi, t0) - pick3(lo, t0)) * (pick3(c, t1) - pick3(lo, t1));
}

// Outward normal velocity on face (a, s) of global cell c (flat index ci)
// of the solution state: boundary faces from the boundary condition,
// faces inside the owning subdomain from the two-point flux of p, faces on
// the skeleton from the owner's Gamma flux (own: the owner's subdomain
// coordinates, sub its index).
__device__ __forceinline__ double state_face_u(const Geo& g, const double* __restrict__ K,
                                               const double* __restrict__ p,
                                               const double* __restrict__ gflux,
                                               const double* __restrict__ bcv, const int c[3],
                                               int ci, const int own[3], int sub, int a, int s) {
  const int q = 2 * a + s;
  int o[3] = {c[0], c[1], c[2]};
  o[a] += s ? 1 : -1;
  K += kaxis(g, a);
  const double kc = K[ci];
  if (off_domain(g, a, c[a], o[a])) {
    const double val = bcv[g.bc_off[q] + bface_index(g, c, a)];
    return g.bc_type[q] ? 2.0 * kc * g.area / g.h * (p[ci] - val) / g.area : val;
  }
  if (o[a] / g.S[a] == own[a]) {
    const int oi = gcell(g, o);
    return g.area * kharm(kc, K[oi]) / g.h * (p[ci] - p[oi]) / g.area;
  }
  int lo[3], hi[3];
  for (int b = 0; b < 3; ++b) {
    lo[b] = (b < g.d) ? own[b] * g.S[b] : 0;
    hi[b] = (b < g.d) ? lo[b] + g.S[b] : 1;
  }
  const int t = side_face_index(g, lo, hi, c, a);
  return gflux[(long long)sub * g.gstride + g.gside_off[q] + t];
}

// Cell coordinates, owning subdomain coordinates and index of cell ci.
__device__ __forceinline__ int cell_owner(const Geo& g, int ci, int c[3], int own[3]) {
  c[0] = ci % g.n[0];
  c[1] = (ci / g.n[0]) % g.n[1];
  c[2] = ci / (g.n[0] * g.n[1]);
  for (int a = 0; a < 3; ++a) own[a] = (a < g.d) ? c[a] / g.S[a] : 0;
  return own[0] + g.M[0] * (own[1] + (g.d == 3 ? g.M[1] * own[2] : 0));
}

// Value of a seed (or interface test function) on the face of side
// `sd.side` of box [lo, hi) touched by global cell c.
__device__ __forceinline__ double seed_value(const Geo& g, const Seed& sd, const int lo[3],
                                             const int hi[3], const int c[3]) {
  const int a = sd.side >> 1;
  if (sd.kind == 0) return 1.0;
  if (sd.kind == 1) {
    const int b = sd.axis;
    const int m = pick3(hi, b) - pick3(lo, b);
    return (2.0 * (pick3(c, b) - pick3(lo, b)) + 1.0) / m - 1.0;
  }
  return side_face_index(g, lo, hi, c, a) == sd.face ? 1.0 : 0.0;
}

// Diagonal of A for a box cell and the couplings to its +axis in-box
// neighbours (T > 0; zero when the neighbour is outside the box).
struct CellCoef {
  double diag;
  double tp[3];
};

__device__ __forceinline__ CellCoef cell_coef(const Geo& g, const Box& B, const double* K,
                                              const int c[3], double beta) {
  CellCoef r;
  r.diag = 0.0;
  r.tp[0] = r.tp[1] = r.tp[2] = 0.0;
  const int ci = gcell(g, c);
  for (int a = 0; a < g.d; ++a) {
    const double* Ka = K + kaxis(g, a);
    const double kc = Ka[ci];
    for (int s = 0; s < 2; ++s) {
      int o[3] = {c[0], c[1], c[2]};
      o[a] += s ? 1 : -1;
      const int kind = face_kind(g, B, c, a, s);
      if (kind == kFaceInterior) {
        const double T = g.area * kharm(kc, Ka[gcell(g, o)]) / g.h;
        r.diag += T;
        if (s) r.tp[a] = T;
      } else if (kind == kFaceRobin) {
        const double b = robin_beta(g, a, kc, Ka[gcell(g, o)], beta);
        r.diag += robin_T(g, kc, b);
      } else if (kind == kFaceDir) {
        r.diag += 2.0 * kc * g.area / g.h;
      }
    }
  }
  return r;
}

}  // namespace mrcm
