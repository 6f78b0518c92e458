// Reverse mode of the MRCM-OS map log K -> (pressure, face velocities), K
// scalar, on the 2-D one-wave-per-box path: the vector-Jacobian product dJ/dlog K for
// given dJ/dp and dJ/d(face velocity), in the FP64 form or the FP32 form
// with FP64 refinement (the precision of the forward solve).
//
// The forward steps are replayed in reverse order (Algorithm 1 backwards):
//   outputs -> smoothing phases (last first; Section 3) -> MRCM-O assembly
//   (eq. addu, addp) -> interface system (eq. int_ujump, int_pjump; solved
//   transposed) -> moments -> basis seeds and particular problems (eq.
//   informed_space, eq111dbar-eq122dbar).
// Every local system A(K) x = b(K, lambda) is symmetric, so its adjoint
// system A mu = xbar reuses the cached block inverses (in the FP32 form:
// the cached FP32 inverses of the scaled matrix, refined in FP64 to the
// forward solve's tolerance, and every forward box solution recomputed by
// the same refinement as the forward pass); the K-dependence of
// A and b enters through the per-face coefficients
//   interior face  T   = |e| K_H / h                 Tbar   = -(mu_c - mu_o)(x_c - x_o)
//   Robin face     T^R = |e| / (h / (2 K_c) + beta)  T^Rbar = mu_c (lambda - x_c)
//   Dirichlet      D   = 2 K_c |e| / h               Dbar   = mu_c (g - x_c)
// and beta = alpha H / K_H (or a constant).  The state before every
// smoothing phase is kept by the forward pass (checkpoints); each phase's
// box solutions are recomputed from them.  Per-cell gradients accumulate
// with atomic adds (boxes overlap).
#include "wave32_common.h"

namespace mrcm {
namespace {

using namespace wave;

// ------------------------------------------------------------- derivatives
struct Dkh {
  double v, da, db;  // K_H = 2ab / (a + b) and its partial derivatives
};

__device__ __forceinline__ Dkh dkh(double a, double b) {
  const double s = a + b, is2 = 1.0 / (s * s);
  return Dkh{2.0 * a * b / s, 2.0 * b * b * is2, 2.0 * a * a * is2};
}

// Robin face between box cell (K = kc) and outside cell (K = ko), normal a.
struct RobinD {
  double bt, TR;            // beta and T^R
  double dbt_c, dbt_o;      // d beta / d K
  double dTR_c, dTR_o;      // d T^R / d K (through K_c directly and through beta)
  double dTR_bt;            // d T^R / d beta
};

__device__ __forceinline__ RobinD robin_d(const Geo& g, int a, double kc, double ko, double beta) {
  RobinD r;
  const double Ha = (a == 0 ? g.S[0] : g.S[1]) * g.h;
  if (g.beta_mode == 1) {
    r.bt = beta;
    r.dbt_c = r.dbt_o = 0.0;
  } else {
    const Dkh k = dkh(kc, ko);
    r.bt = beta * Ha / k.v;
    const double q = -beta * Ha / (k.v * k.v);
    r.dbt_c = q * k.da;
    r.dbt_o = q * k.db;
  }
  const double den = g.h + 2.0 * kc * r.bt, iden2 = 1.0 / (den * den);
  r.TR = g.area * 2.0 * kc / den;
  r.dTR_bt = -g.area * 4.0 * kc * kc * iden2;
  r.dTR_c = g.area * 2.0 * g.h * iden2 + r.dTR_bt * r.dbt_c;
  r.dTR_o = r.dTR_bt * r.dbt_o;
  return r;
}

__device__ __forceinline__ void kadd(double* Kb, const Geo& g, int x, int y, double v) {
  if (v != 0.0) atomicAdd(Kb + x + g.n[0] * y, v);
}

// Gradient terms of the box matrix and of the K-dependent right-hand-side
// coefficients for nrhs solutions x_k and adjoint solutions mu_k (LDS,
// stride nc), Robin data lam(k, q, t) and Dirichlet values gval(q, t):
//   K_bar += -mu^T (dA/dK) x + mu^T (db/dK)      (summed over k)
// and lambda_bar(k, q, t) = T^R mu_c reported through lbar(k, q, t, value).
template <int NT, typename Lam, typename GVal, typename LBar>
__device__ __forceinline__ void box_matrix_adjoint(const Geo& g, const Box& B, const BoxLds& s,
                                                   const double* x, const double* mu, int nrhs,
                                                   double beta, Lam lam, GVal gval, LBar lbar,
                                                   double* Kb) {
  const int m0 = s.m0, m1 = s.m1, nc = m0 * m1;
  const int tid = threadIdx.x % NT;
  // interior faces: (c, c + 1) along x and (c, c + m0) along y
#pragma unroll 1
  for (int u = tid; u < 2 * nc; u += NT) {
    const int a = u >= nc, c = a ? u - nc : u;
    const int xl = c % m0, yl = c / m0;
    if (a == 0 ? xl + 1 >= m0 : yl + 1 >= m1) continue;
    const int o = a == 0 ? c + 1 : c + m0;
    double tb = 0.0;
    for (int k = 0; k < nrhs; ++k)
      tb -= (mu[k * nc + c] - mu[k * nc + o]) * (x[k * nc + c] - x[k * nc + o]);
    const int gx = B.lo[0] + xl, gy = B.lo[1] + yl;
    const Dkh kk = dkh(kat(s, B, gx, gy, a), kat(s, B, gx + (a == 0), gy + (a == 1), a));
    const double f = tb * g.area / g.h;
    kadd(Kb, g, gx, gy, f * kk.da);
    kadd(Kb, g, gx + (a == 0), gy + (a == 1), f * kk.db);
  }
  // faces of the box sides: Robin (interior of the domain) or Dirichlet
  const int ns = 2 * (m0 + m1);
#pragma unroll 1
  for (int u = tid; u < ns; u += NT) {
    const int q = u < 2 * m1 ? (u < m1 ? 0 : 1) : (u < 2 * m1 + m0 ? 2 : 3);
    const int t = u - (q == 0 ? 0 : q == 1 ? m1 : q == 2 ? 2 * m1 : 2 * m1 + m0);
    const int a = q >> 1, sd = q & 1;
    const int xl = a == 0 ? (sd ? m0 - 1 : 0) : t, yl = a == 1 ? (sd ? m1 - 1 : 0) : t;
    const int gx = B.lo[0] + xl, gy = B.lo[1] + yl;
    const int ox = gx + (a == 0 ? (sd ? 1 : -1) : 0), oy = gy + (a == 1 ? (sd ? 1 : -1) : 0);
    const int c = xl + m0 * yl;
    const double kc = kat(s, B, gx, gy, a);
    const bool dom = off_domain(g, a, a == 0 ? gx : gy, a == 0 ? ox : oy);
    if (dom) {
      if (!g.bc_type[q]) continue;
      const double gv = gval(q, t);
      double db = 0.0;
      for (int k = 0; k < nrhs; ++k) db += mu[k * nc + c] * (gv - x[k * nc + c]);
      kadd(Kb, g, gx, gy, db * 2.0 * g.area / g.h);
      continue;
    }
    const RobinD r = robin_d(g, a, kc, kat(s, B, ox, oy, a), beta);
    double trb = 0.0;
    for (int k = 0; k < nrhs; ++k) {
      const double m = mu[k * nc + c];
      trb += m * (lam(k, q, t) - x[k * nc + c]);
      lbar(k, q, t, r.TR * m);
    }
    kadd(Kb, g, gx, gy, trb * r.dTR_c);
    kadd(Kb, g, ox, oy, trb * r.dTR_o);
  }
}

// ------------------------------------------------------------------ outputs
// pb = dJ/dp - mean (pure Neumann) plus the face-velocity terms; gfb on the
// Gamma faces; Kb from the two-point and Dirichlet face velocities.  Gather
// form: every cell collects its own and its neighbours' face terms.
__global__ void k_adj_out(Geo g, const double* __restrict__ K, const double* __restrict__ p,
                          const double* __restrict__ bcv, const double* __restrict__ dJdp,
                          const double* __restrict__ dJdf, const double* __restrict__ meanp,
                          double* __restrict__ pb, double* __restrict__ gfb, double* __restrict__ Kb) {
  const int ci = blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= g.ncells) return;
  const int cx = ci % g.n[0], cy = ci / g.n[0];
  const int ix = cx / g.S[0], iy = cy / g.S[1];
  const int sub = ix + g.M[0] * iy;
  double vp = dJdp ? dJdp[ci] - (g.neumann ? *meanp : 0.0) : 0.0;
  double vk = 0.0;
  const double kc = K[ci], pc = p[ci];
  if (dJdf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = q >> 1, sd = q & 1;
      const int ox = cx + (a == 0 ? (sd ? 1 : -1) : 0), oy = cy + (a == 1 ? (sd ? 1 : -1) : 0);
      const double ub = dJdf[(long long)ci * 4 + q];
      if (off_domain(g, a, a == 0 ? cx : cy, a == 0 ? ox : oy)) {
        if (g.bc_type[q]) {
          const int off = q == 0 ? g.bc_off[0] : q == 1 ? g.bc_off[1] : q == 2 ? g.bc_off[2] : g.bc_off[3];
          const int c3[3] = {cx, cy, 0};
          const double val = bcv[off + bface_index(g, c3, a)];
          vp += ub * 2.0 * kc / g.h;
          vk += ub * 2.0 * (pc - val) / g.h;
        }
        continue;
      }
      const int oi = ox + g.n[0] * oy;
      const bool same = (a == 0 ? ox / g.S[0] == ix : oy / g.S[1] == iy);
      if (same) {
        // u_c = K_H (p_c - p_o) / h on this face and u_o = -u_c on the
        // neighbour's face q ^ 1
        const double ubo = dJdf[(long long)oi * 4 + (q ^ 1)];
        const Dkh kk = dkh(kc, K[oi]);
        vp += (ub - ubo) * kk.v / g.h;
        vk += (ub - ubo) * (pc - p[oi]) / g.h * kk.da;
      } else {
        const int go = q == 0 ? g.gside_off[0] : q == 1 ? g.gside_off[1] : q == 2 ? g.gside_off[2] : g.gside_off[3];
        const int t = a == 0 ? cy - iy * g.S[1] : cx - ix * g.S[0];
        gfb[(long long)sub * g.gstride + go + t] = ub;
      }
    }
  }
  pb[ci] = vp;
  Kb[ci] = vk;
}

__global__ void k_adj_mean(const double* __restrict__ v, int n, double* __restrict__ out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += v[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0] / n;
}

// --------------------------------------------------------------- smoothing
constexpr int kAdjNT = 256;

// Doubles before the adjoint's own arrays in the FP32 forms' LDS: the FP32
// smoothing box (carve_smooth + carve_smooth_r), a refinement box of nrhs
// right-hand sides (carve_r), each rounded up to 16 bytes.
__host__ __device__ inline size_t adj_smooth32_off(int m0, int m1) {
  return (smooth32_lds_bytes(m0, m1) + 15) / 16 * 2;
}
__host__ __device__ inline size_t adj_box32_off(int m0, int m1, int nrhs) {
  return (boxr_bytes(m0, m1, nrhs, nrhs) + 15) / 16 * 2;
}

// One right-hand side in s.X solved by one wave with the two-ended sweep of
// the cached factors (forward inverses below the meeting block, backward
// inverses above it and Z_m): the same arithmetic as the forward smoothing
// step, so the reverse pass recomputes the forward state exactly.
__device__ __forceinline__ void box_solve(const Box& B, const double* Wf, const double* Wt,
                                          const BoxLds& s, double* z) {
  double w[RING][HB], zm[HB];
  wload_block(block_src(Wt, B.nb, B.nblk), B.nblk / 2, zm);
  sweep_twisted<64>(B, Wf, Wt, s, z, w, zm);
}

// One colour phase in reverse.  p_in / gf_in: the state before the phase.
// F32: the FP32 form (fac, fact and tcoup unused; the FP32 factors and the
// refinement settings in rf).
template <bool F32>
__global__ void __launch_bounds__(kAdjNT) k_adj_smooth(Geo g, const Box* __restrict__ boxes,
                                                       const int* __restrict__ members,
                                                       const double* __restrict__ K,
                                                       const double* __restrict__ f,
                                                       const double* __restrict__ bcv, double beta,
                                                       const double* __restrict__ fac,
                                                       const double* __restrict__ fact,
                                                       const double* __restrict__ tcoup, Adj32 rf,
                                                       const double* __restrict__ p_in,
                                                       const double* __restrict__ gf_in,
                                                       double* __restrict__ pb,
                                                       double* __restrict__ gfb,
                                                       double* __restrict__ Kb) {
  constexpr int NT = kAdjNT;
  extern __shared__ __align__(16) double dsm[];
  __shared__ WaveSmemF sm32;
  const Box B = boxes[members[blockIdx.x]];
  SmoothLds r = carve_smooth(dsm, B);
  const int m0 = r.b.m0, m1 = r.b.m1, nc = m0 * m1, ns = 2 * (m0 + m1);
  BoxR R{};
  if (F32) R = carve_smooth_r(dsm, r);
  double* xs = dsm + (F32 ? adj_smooth32_off(m0, m1) : smooth_lds_doubles(m0, m1));  // forward solution
  double* mu = xs + nc;                             // adjoint right-hand side / solution
  double* lb = mu + nc;                             // lambda_bar per box-side face
  const int tid = threadIdx.x;
  if (F32 && tid == 0) sm32.flag = 0;
  // (a) forward solution of this box from the checkpointed state (the
  // forward smoothing step's arithmetic)
  if (F32) {
    stage_smooth<NT>(g, B, r, K, p_in, f, gf_in, bcv, nullptr);
    __syncthreads();
    smooth_rhs<NT>(g, B, r, beta, R.Bv);
    coef_box<NT>(g, B, beta, R.b);
    scale_box<NT>(B, R);
    if (tid < 64) {
      double om = 0.0;
      const int it = refine<true>(g, B, R, rf.fac + B.fac, 1, nullptr, beta, rf.tol, rf.max_refine, om, sm32);
      record_refine(it, om, rf.iters, rf.resid);
    }
  } else {
    stage_smooth<NT>(g, B, r, K, p_in, f, gf_in, bcv, tcoup);
    __syncthreads();
    smooth_rhs<NT>(g, B, r, beta, r.b.X);
    if (tid < 64) box_solve(B, fac + B.fac, fact + B.fac, r.b, r.b.Z);
  }
  __syncthreads();
  for (int e = tid; e < nc; e += NT) {
    xs[e] = r.b.X[e];
    mu[e] = 0.0;
  }
  for (int e = tid; e < ns; e += NT) lb[e] = 0.0;
  __syncthreads();
  // (b) adjoint of the outputs: p on Omega_i and Omega_i's Gamma fluxes
  int olo[3], ohi[3];
  womega(g, B.sub, olo, ohi);
  const int ncell_o = g.S[0] * g.S[1];
  for (int t = tid; t < ncell_o; t += NT) {
    const int cx = olo[0] + t % g.S[0], cy = olo[1] + t / g.S[0];
    const int ci = cx + g.n[0] * cy;
    mu[bloc(B, r.b, cx, cy)] += pb[ci];
    pb[ci] = 0.0;
  }
  __syncthreads();
  // one pass per side of Omega_i: with a subdomain one cell thick along a,
  // both sides of that axis add to the same cells
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    const int a = q >> 1, so = q & 1;
    const int nf = a == 0 ? g.S[1] : g.S[0];
    for (int t = tid; t < nf; t += NT) {
      if (wneighbor(g, B.sub, q) < 0) continue;
      int cx, cy;
      wgface(olo, ohi, q, t, cx, cy);
      const int ox = cx + (a == 0 ? (so ? 1 : -1) : 0), oy = cy + (a == 1 ? (so ? 1 : -1) : 0);
      const int go = q == 0 ? g.gside_off[0] : q == 1 ? g.gside_off[1] : q == 2 ? g.gside_off[2] : g.gside_off[3];
      double* gp = gfb + (long long)B.sub * g.gstride + go + t;
      const double ub = *gp;
      *gp = 0.0;
      if (ub == 0.0) continue;
      const double kc = kat(r.b, B, cx, cy, a), ko = kat(r.b, B, ox, oy, a);
      const int c = bloc(B, r.b, cx, cy);
      if (win_box(B, ox, oy)) {
        const int o = bloc(B, r.b, ox, oy);
        const Dkh kk = dkh(kc, ko);
        mu[c] += ub * kk.v / g.h;
        mu[o] -= ub * kk.v / g.h;
        const double dx = (xs[c] - xs[o]) / g.h;
        kadd(Kb, g, cx, cy, ub * dx * kk.da);
        kadd(Kb, g, ox, oy, ub * dx * kk.db);
      } else {
        // no overlap: u = T^R (x_c - lambda) / |e| with the staged lambda
        const RobinD rd = robin_d(g, a, kc, ko, beta);
        const double lam = lambda_s(g, B, r, rd.bt, cx, cy, a, so);
        mu[c] += ub * rd.TR / g.area;
        const int sf = side_off(r.b, q) + (a == 0 ? cy - B.lo[1] : cx - B.lo[0]);
        lb[sf] -= ub * rd.TR / g.area;
        const double trb = ub * (xs[c] - lam) / g.area;
        kadd(Kb, g, cx, cy, trb * rd.dTR_c);
        kadd(Kb, g, ox, oy, trb * rd.dTR_o);
        // lambda's own beta is the face's beta: its K-dependence is carried
        // with lambda_bar below
      }
    }
    __syncthreads();
  }
  // (c) adjoint solve A mu = xbar (A symmetric: cached inverses)
  if (F32) {
    for (int e = tid; e < nc; e += NT) R.Bv[e] = mu[e];
    __syncthreads();
    if (tid < 64) {
      double om = 0.0;
      const int it = refine<true>(g, B, R, rf.fac + B.fac, 1, nullptr, beta, rf.tol, rf.max_refine, om, sm32);
      record_refine(it, om, rf.iters, rf.resid);
    }
    __syncthreads();
    for (int e = tid; e < nc; e += NT) mu[e] = R.b.X[e];
  } else {
    BoxLds sm = r.b;
    sm.X = mu;
    if (tid < 64) box_solve(B, fac + B.fac, fact + B.fac, sm, r.b.Z);
  }
  __syncthreads();
  // (d) K terms of the box matrix and right-hand side; lambda_bar of the
  // Robin faces
  box_matrix_adjoint<NT>(
      g, B, r.b, xs, mu, 1, beta,
      [&](int, int q, int t) {
        const int a = q >> 1, sd = q & 1;
        const int cx = a == 0 ? (sd ? B.hi[0] - 1 : B.lo[0]) : B.lo[0] + t;
        const int cy = a == 1 ? (sd ? B.hi[1] - 1 : B.lo[1]) : B.lo[1] + t;
        const int ox = cx + (a == 0 ? (sd ? 1 : -1) : 0), oy = cy + (a == 1 ? (sd ? 1 : -1) : 0);
        const RobinD rd = robin_d(g, a, kat(r.b, B, cx, cy, a), kat(r.b, B, ox, oy, a), beta);
        return lambda_s(g, B, r, rd.bt, cx, cy, a, sd);
      },
      [&](int q, int t) { return r.BC[side_off(r.b, q) + t]; },
      [&](int, int q, int t, double v) { atomicAdd(lb + side_off(r.b, q) + t, v); }, Kb);
  __syncthreads();
  // (e) lambda = lambda(p_in, gf_in, K) on every Robin face of the box
  for (int u = tid; u < ns; u += NT) {
    const double lbar = lb[u];
    if (lbar == 0.0) continue;
    const int q = u < 2 * m1 ? (u < m1 ? 0 : 1) : (u < 2 * m1 + m0 ? 2 : 3);
    const int t = u - side_off(r.b, q);
    const int a = q >> 1, sd = q & 1;
    const int cx = a == 0 ? (sd ? B.hi[0] - 1 : B.lo[0]) : B.lo[0] + t;
    const int cy = a == 1 ? (sd ? B.hi[1] - 1 : B.lo[1]) : B.lo[1] + t;
    const int ox = cx + (a == 0 ? (sd ? 1 : -1) : 0), oy = cy + (a == 1 ? (sd ? 1 : -1) : 0);
    const int ti = tile_at(r.b, B, cx, cy), to = tile_at(r.b, B, ox, oy);
    const double kc = ktile(r.b, a)[ti], ko = ktile(r.b, a)[to];
    const RobinD rd = robin_d(g, a, kc, ko, beta);
    const int ci = cx + g.n[0] * cy, oi = ox + g.n[0] * oy;
    if (g.l > 0) {
      // lambda = -beta u + p_c - u h / (2 K_c),  u = K_H (p_c - p_o) / h
      const Dkh kk = dkh(kc, ko);
      const double pc = r.P[ti], po = r.P[to];
      const double uu = kk.v * (pc - po) / g.h;
      const double dlu = -rd.bt - g.h / (2.0 * kc);
      atomicAdd(pb + ci, lbar * (1.0 + dlu * kk.v / g.h));
      atomicAdd(pb + oi, -lbar * dlu * kk.v / g.h);
      const double du_c = (pc - po) / g.h * kk.da, du_o = (pc - po) / g.h * kk.db;
      kadd(Kb, g, cx, cy, lbar * (dlu * du_c + uu * g.h / (2.0 * kc * kc) - uu * rd.dbt_c));
      kadd(Kb, g, ox, oy, lbar * (dlu * du_o - uu * rd.dbt_o));
    } else {
      // lambda = beta u_j + p_o - u_j h / (2 K_o), u_j the neighbour's flux
      const int j = B.sub + (a == 0 ? (sd ? 1 : -1) : (sd ? g.M[0] : -g.M[0]));
      const int jx = j % g.M[0], jy = j / g.M[0];
      const int tj = a == 0 ? cy - jy * g.S[1] : cx - jx * g.S[0];
      const int go = q == 0 ? g.gside_off[1] : q == 1 ? g.gside_off[0] : q == 2 ? g.gside_off[3] : g.gside_off[2];
      const long long gj = (long long)j * g.gstride + go + tj;
      const double uj = r.GF[u];
      atomicAdd(gfb + gj, lbar * (rd.bt - g.h / (2.0 * ko)));
      atomicAdd(pb + oi, lbar);
      kadd(Kb, g, ox, oy, lbar * (uj * g.h / (2.0 * ko * ko) + uj * rd.dbt_o));
      kadd(Kb, g, cx, cy, lbar * uj * rd.dbt_c);
      (void)ci;
    }
  }
  if (F32) {
    __syncthreads();
    if (tid == 0 && sm32.flag) atomicOr(rf.flags, sm32.flag);
  }
}

// ---------------------------------------------------------- MRCM-O assembly
// Xbar_k = sum_t pb(cell t of Omega_i) P_k(t) + sum gfb_i tr_u_k; one
// workgroup per seed.  Also tr_ub = X_k gfb_i (initialises tr_ub).
__global__ void __launch_bounds__(256) k_adj_combine(Geo g, const int* __restrict__ seed_sub,
                                                     const double* __restrict__ X,
                                                     const double* __restrict__ Pk,
                                                     const double* __restrict__ tr_u,
                                                     const double* __restrict__ pb,
                                                     const double* __restrict__ gfb,
                                                     double* __restrict__ Xb,
                                                     double* __restrict__ tr_ub) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  const int sub = seed_sub[k];
  const int ncell_o = g.S[0] * g.S[1];
  const int ix = sub % g.M[0], iy = sub / g.M[0];
  double acc = 0.0;
  for (int t = threadIdx.x; t < ncell_o; t += 256) {
    const int cx = ix * g.S[0] + t % g.S[0], cy = iy * g.S[1] + t / g.S[0];
    acc += pb[cx + g.n[0] * cy] * Pk[(long long)k * ncell_o + t];
  }
  for (int t = threadIdx.x; t < g.gstride; t += 256) {
    const double v = gfb[(long long)sub * g.gstride + t];
    acc += v * tr_u[(long long)k * g.gstride + t];
    tr_ub[(long long)k * g.gstride + t] = X[k] * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) Xb[k] = red[0];
}

// ------------------------------------------------------------------ moments
// Adjoint of the moment equations for the solution nu of G^T nu = Xbar:
// Gbar = -nu X^T on the structural entries, rbar = nu.  One workgroup per
// interface; threads over (side, seed or particular, face), rows in a loop
// (each trace entry belongs to one interface, so no atomics).
__global__ void k_adj_moments(Geo g, const Iface* __restrict__ ifc, const Seed* __restrict__ basis,
                              const int* __restrict__ seed_off, const double* __restrict__ X,
                              const double* __restrict__ nu, const double* __restrict__ tr_u,
                              const double* __restrict__ tr_beta, double* __restrict__ tr_ub,
                              double* __restrict__ tr_phib, double* __restrict__ tr_betab,
                              double* __restrict__ ubarb, double* __restrict__ pibarb) {
  const Iface F = ifc[blockIdx.x];
  const int qi = 2 * F.axis + 1, qj = 2 * F.axis;
  const int ni = seed_off[F.i + 1] - seed_off[F.i];
  const int nj = seed_off[F.j + 1] - seed_off[F.j];
  int ilo[3], ihi[3];
  womega(g, F.i, ilo, ihi);
  const int nf = F.axis == 0 ? g.S[1] : g.S[0];
  const int per_t = ni + nj + 2;  // seeds of i, seeds of j, particular of i and of j
  for (int w = threadIdx.x; w < per_t * nf; w += blockDim.x) {
    const int e = w / nf, t = w % nf;
    int cx, cy;
    wgface(ilo, ihi, qi, t, cx, cy);
    const int c[3] = {cx, cy, 0};
    const bool is_part = e >= ni + nj;
    const bool side_i = is_part ? e == ni + nj : e < ni;
    const int sub = side_i ? F.i : F.j;
    const int q = side_i ? qi : qj;
    const long long bface = (long long)sub * g.gstride + g.gside_off[q] + t;
    const int col = is_part ? -1 : seed_off[sub] + (side_i ? e : e - ni);
    const long long tface = (long long)col * g.gstride + g.gside_off[q] + t;
    double gu = 0.0, gphi = 0.0, gbeta = 0.0, gub = 0.0, gpb = 0.0;
    for (int rr = 0; rr < 2 * F.nbasis; ++rr) {
      const int row = F.row0 + rr;
      if (g.neumann && row == 0) continue;  // gauge row: constant entries
      const int kind = rr / F.nbasis;       // 0 flux, 1 pressure
      const Seed mu = basis[F.basis0 + rr % F.nbasis];
      const double wt = g.area * seed_value(g, mu, ilo, ihi, c);
      const double sg = (kind == 1 && !side_i) ? -1.0 : 1.0;
      const double v = nu[row];
      if (is_part) {
        // r_row = -sum sg w (ubar or pibar)
        if (kind == 0) gub -= sg * wt * v;
        else gpb -= sg * wt * v;
      } else {
        const double gb = -v * X[col] * sg * wt;  // Gbar(row, col) sg w
        if (kind == 0) {
          gu += gb;
        } else {
          gu += gb * tr_beta[bface];
          gphi += gb;
          gbeta += gb * tr_u[tface];
        }
      }
    }
    if (is_part) {
      ubarb[bface] += gub;
      pibarb[bface] = gpb;
    } else {
      tr_ub[tface] += gu;
      tr_phib[tface] = gphi;
      atomicAdd(tr_betab + bface, gbeta);
    }
  }
}

// ------------------------------------------------------------ seeds (basis)
// Per oversampled box: recompute the seed solutions P_k, form their adjoint
// right-hand sides (Omega_i restriction and Gamma traces u, phi, beta),
// solve with the cached inverses and accumulate the K terms.  F32: the
// FP32 form (fac and fact unused).
template <bool F32>
__global__ void __launch_bounds__(64) k_adj_basis(Geo g, const Box* __restrict__ boxes,
                                                  const Seed* __restrict__ seeds,
                                                  const double* __restrict__ K, double beta,
                                                  const double* __restrict__ fac,
                                                  const double* __restrict__ fact, Adj32 rf,
                                                  const double* __restrict__ X,
                                                  const double* __restrict__ pb,
                                                  const double* __restrict__ tr_u,
                                                  const double* __restrict__ tr_ub,
                                                  const double* __restrict__ tr_phib,
                                                  const double* __restrict__ tr_betab,
                                                  double* __restrict__ Kb) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ WaveSmemF sm32;
  const Box B = boxes[blockIdx.x];
  const int L = lane_id();
  const int nrhs = B.nrhs;
  BoxR R{};
  BoxLds s;
  double* xs;  // nrhs x nc forward solutions
  if (F32) {
    R = carve_r(dsm, B, max(nrhs, 1), max(nrhs, 1));
    s = R.b;
    xs = dsm + adj_box32_off(s.m0, s.m1, max(nrhs, 1));
  } else {
    s = carve(dsm, B, nrhs);
    xs = dsm + box_lds_doubles(s.m0, s.m1, nrhs);
  }
  const int nc = B.ncell;
  if (F32 && L == 0) sm32.flag = 0;
  load_box(g, B, K, beta, s);
  auto seed_lam = [&](int k, int q, int t) -> double {
    const Seed sd = seeds[B.seed0 + k];
    if (sd.side != q) return 0.0;
    const int a = q >> 1, so = q & 1;
    int c[3];
    c[0] = a == 0 ? (so ? B.hi[0] - 1 : B.lo[0]) : B.lo[0] + t;
    c[1] = a == 1 ? (so ? B.hi[1] - 1 : B.lo[1]) : B.lo[1] + t;
    c[2] = 0;
    return seed_value(g, sd, B.lo, B.hi, c);
  };
  const double* Wf = fac + B.fac;
  const double* Wt = fact + B.fac;
  if (F32) {
    // the forward basis kernel's refinement of the seed problems
    scale_box(B, R);
    if (nrhs > 0) {
      double om = 0.0;
      const int it = refine<false>(g, B, R, rf.fac + B.fac, nrhs, seeds, beta, rf.tol, rf.max_refine, om, sm32);
      record_refine(it, om, rf.iters, rf.resid);
    }
  } else {
    // seed right-hand sides (T^R times the seed on its side)
    for (int e = L; e < nrhs * nc; e += 64) s.X[e] = 0.0;
    wsync();
    for (int k = 0; k < nrhs; ++k) {
      const Seed sd = seeds[B.seed0 + k];
      const int a = sd.side >> 1, so = sd.side & 1;
      const int nf = a == 0 ? s.m1 : s.m0;
      for (int t = L; t < nf; t += 64) {
        const int cx = a == 0 ? (so ? B.hi[0] - 1 : B.lo[0]) : B.lo[0] + t;
        const int cy = a == 1 ? (so ? B.hi[1] - 1 : B.lo[1]) : B.lo[1] + t;
        const int ox = cx + (a == 0 ? (so ? 1 : -1) : 0), oy = cy + (a == 1 ? (so ? 1 : -1) : 0);
        const RobinD rd = robin_d(g, a, kat(s, B, cx, cy, a), kat(s, B, ox, oy, a), beta);
        s.X[k * nc + bloc(B, s, cx, cy)] = rd.TR * seed_lam(k, sd.side, t);
      }
    }
    wsync();
    twisted_cached(B, Wf, Wt, nrhs, s);
  }
  wsync();
  for (int e = L; e < nrhs * nc; e += 64) {
    xs[e] = s.X[e];
    s.X[e] = 0.0;
  }
  wsync();
  // adjoint right-hand sides: Omega_i cells (combine) and Gamma traces
  int olo[3], ohi[3];
  womega(g, B.sub, olo, ohi);
  const int ncell_o = g.S[0] * g.S[1];
  for (int e = L; e < nrhs * ncell_o; e += 64) {
    const int k = e / ncell_o, t = e % ncell_o;
    const int cx = olo[0] + t % g.S[0], cy = olo[1] + t / g.S[0];
    s.X[k * nc + bloc(B, s, cx, cy)] += X[B.seed0 + k] * pb[cx + g.n[0] * cy];
  }
  wsync();
  // one pass per side of Omega_i: with a subdomain one cell thick along a,
  // both sides of that axis add to the same cells
  for (int q = 0; q < 4; ++q) {
    const int a = q >> 1, so = q & 1;
    const int nf = a == 0 ? g.S[1] : g.S[0];
    for (int e = L; e < nrhs * nf; e += 64) {
      const int k = e / nf, t = e % nf;
      if (wneighbor(g, B.sub, q) < 0) continue;
      const int go = q == 0 ? g.gside_off[0] : q == 1 ? g.gside_off[1] : q == 2 ? g.gside_off[2] : g.gside_off[3];
      const long long tf = (long long)(B.seed0 + k) * g.gstride + go + t;
      const long long bf = (long long)B.sub * g.gstride + go + t;
      const double uub = tr_ub[tf], phib = tr_phib[tf], betab = k == 0 ? tr_betab[bf] : 0.0;
      int cx, cy;
      wgface(olo, ohi, q, t, cx, cy);
      const int ox = cx + (a == 0 ? (so ? 1 : -1) : 0), oy = cy + (a == 1 ? (so ? 1 : -1) : 0);
      const double kc = kat(s, B, cx, cy, a), ko = kat(s, B, ox, oy, a);
      const RobinD rd = robin_d(g, a, kc, ko, beta);
      const int c = bloc(B, s, cx, cy);
      const double xc = xs[k * nc + c];
      const double uval = tr_u[tf];
      // phi = -beta u + x_c - u h / (2 K_c);  beta = beta(K_c, K_o)
      const double ut = uub + phib * (-rd.bt - g.h / (2.0 * kc));
      double* xb = s.X + k * nc;
      xb[c] += phib;
      double kcb = phib * uval * g.h / (2.0 * kc * kc);
      const double btb = betab - phib * uval;
      double kob = 0.0;
      kcb += btb * rd.dbt_c;
      kob += btb * rd.dbt_o;
      if (win_box(B, ox, oy)) {
        const int o = bloc(B, s, ox, oy);
        const Dkh kk = dkh(kc, ko);
        xb[c] += ut * kk.v / g.h;
        xb[o] -= ut * kk.v / g.h;
        const double dx = (xc - xs[k * nc + o]) / g.h;
        kcb += ut * dx * kk.da;
        kob += ut * dx * kk.db;
      } else {
        // no overlap: u = T^R (x_c - lambda_seed) / |e|
        const double lam = seed_lam(k, q, a == 0 ? cy - B.lo[1] : cx - B.lo[0]);
        xb[c] += ut * rd.TR / g.area;
        const double trb = ut * (xc - lam) / g.area;
        kcb += trb * rd.dTR_c;
        kob += trb * rd.dTR_o;
      }
      kadd(Kb, g, cx, cy, kcb);
      kadd(Kb, g, ox, oy, kob);
    }
    wsync();
  }
  // adjoint solves with the cached factors (A symmetric)
  if (F32) {
    for (int e = L; e < nrhs * nc; e += 64) R.Bv[e] = s.X[e];
    wsync();
    if (nrhs > 0) {
      double om = 0.0;
      const int it = refine<false>(g, B, R, rf.fac + B.fac, nrhs, nullptr, beta, rf.tol, rf.max_refine, om, sm32);
      record_refine(it, om, rf.iters, rf.resid);
    }
  } else {
    twisted_cached(B, Wf, Wt, nrhs, s);
  }
  wsync();
  box_matrix_adjoint<64>(
      g, B, s, xs, s.X, nrhs, beta, seed_lam, [](int, int) { return 0.0; },
      [](int, int, int, double) {}, Kb);
  if (F32) {
    wsync();
    if (L == 0 && sm32.flag) atomicOr(rf.flags, sm32.flag);
  }
}

// --------------------------------------------------------------- particular
// Per subdomain: the particular solution pbar is stored; its adjoint
// right-hand side collects pb on Omega_i and the Gamma traces ubar, pibar.
// F32: the FP32 form (fac unused).
template <bool F32>
__global__ void __launch_bounds__(64) k_adj_particular(Geo g, const Box* __restrict__ boxes,
                                                       const double* __restrict__ K,
                                                       const double* __restrict__ bcv, double beta,
                                                       const double* __restrict__ fac, Adj32 rf,
                                                       const double* __restrict__ pbar,
                                                       const double* __restrict__ pb,
                                                       const double* __restrict__ ubarb,
                                                       const double* __restrict__ pibarb,
                                                       double* __restrict__ Kb) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ WaveSmemF sm32;
  const Box B = boxes[blockIdx.x];
  const int L = lane_id();
  BoxR R{};
  BoxLds s;
  double* xs;
  if (F32) {
    R = carve_r(dsm, B, 1, 1);
    s = R.b;
    xs = dsm + adj_box32_off(s.m0, s.m1, 1);
  } else {
    s = carve(dsm, B, 1);
    // the single-right-hand-side sweep stages through 2 x NBW doubles at s.Z
    xs = dsm + box_lds_doubles(s.m0, s.m1, 1) + NBW;
  }
  const int nc = B.ncell;
  double* bc = xs + nc;  // boundary value per box-side face
  if (F32 && L == 0) sm32.flag = 0;
  load_box(g, B, K, beta, s);
  if (F32) scale_box(B, R);
  const int m0 = s.m0, m1 = s.m1, ns = 2 * (m0 + m1);
  for (int u = L; u < ns; u += 64) {
    const int q = u < 2 * m1 ? (u < m1 ? 0 : 1) : (u < 2 * m1 + m0 ? 2 : 3);
    const int t = u - side_off(s, q);
    const int a = q >> 1, sd = q & 1;
    const int cx = a == 0 ? (sd ? B.hi[0] - 1 : B.lo[0]) : B.lo[0] + t;
    const int cy = a == 1 ? (sd ? B.hi[1] - 1 : B.lo[1]) : B.lo[1] + t;
    const int o = (a == 0 ? cx : cy) + (sd ? 1 : -1);
    const bool dom = off_domain(g, a, a == 0 ? cx : cy, o);
    const int off = q == 0 ? g.bc_off[0] : q == 1 ? g.bc_off[1] : q == 2 ? g.bc_off[2] : g.bc_off[3];
    const int c3[3] = {cx, cy, 0};
    bc[u] = dom ? bcv[off + bface_index(g, c3, a)] : 0.0;
  }
  for (int e = L; e < nc; e += 64) {
    xs[e] = pbar[(long long)B.sub * nc + e];
    const int cx = B.lo[0] + e % m0, cy = B.lo[1] + e / m0;
    s.X[e] = pb[cx + g.n[0] * cy];
  }
  wsync();
  for (int q = 0; q < 4; ++q) {  // one pass per side, as above
    const int a = q >> 1, so = q & 1;
    const int nf = a == 0 ? g.S[1] : g.S[0];
    for (int t = L; t < nf; t += 64) {
      if (wneighbor(g, B.sub, q) < 0) continue;
      const int go = q == 0 ? g.gside_off[0] : q == 1 ? g.gside_off[1] : q == 2 ? g.gside_off[2] : g.gside_off[3];
      const long long bf = (long long)B.sub * g.gstride + go + t;
      int cx, cy;
      wgface(B.lo, B.hi, q, t, cx, cy);
      const int ox = cx + (a == 0 ? (so ? 1 : -1) : 0), oy = cy + (a == 1 ? (so ? 1 : -1) : 0);
      const double kc = kat(s, B, cx, cy, a), ko = kat(s, B, ox, oy, a);
      const RobinD rd = robin_d(g, a, kc, ko, beta);
      const int c = bloc(B, s, cx, cy);
      // ubar = T^R pbar_c / |e|, pibar = beta ubar
      const double ub = ubarb[bf], pib = pibarb[bf];
      const double uval = rd.TR * xs[c] / g.area;
      const double ut = ub + pib * rd.bt;
      s.X[c] += ut * rd.TR / g.area;
      const double trb = ut * xs[c] / g.area;
      const double btb = pib * uval;
      kadd(Kb, g, cx, cy, trb * rd.dTR_c + btb * rd.dbt_c);
      kadd(Kb, g, ox, oy, trb * rd.dTR_o + btb * rd.dbt_o);
    }
    wsync();
  }
  if (F32) {
    for (int e = L; e < nc; e += 64) R.Bv[e] = s.X[e];
    wsync();
    double om = 0.0;
    const int it = refine<true>(g, B, R, rf.fac + B.fac, 1, nullptr, beta, rf.tol, rf.max_refine, om, sm32);
    record_refine(it, om, rf.iters, rf.resid);
  } else {
    sweep1(B, fac + B.fac, s, s.Z);
  }
  box_matrix_adjoint<64>(
      g, B, s, xs, s.X, 1, beta, [](int, int, int) { return 0.0; },
      [&](int q, int t) { return bc[side_off(s, q) + t]; }, [](int, int, int, double) {}, Kb);
  if (F32) {
    wsync();
    if (L == 0 && sm32.flag) atomicOr(rf.flags, sm32.flag);
  }
}

__global__ void k_adj_logk(const double* __restrict__ K, const double* __restrict__ Kb, int n,
                           double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = K[i] * Kb[i];
}

// Transposed scatter of the band system into the layer blocks: G^T's rows
// are G's columns.  The right-hand side is indexed by G's columns.
__global__ void k_bcr_scatter_t(const double* __restrict__ RB, const double* __restrict__ rhs,
                                int n, int kl, int ku, const int* __restrict__ row_lvl,
                                const int* __restrict__ row_loc, const int* __restrict__ col_lvl,
                                const int* __restrict__ col_loc, int M, int bp,
                                double* __restrict__ pool, double* __restrict__ vec) {
  const int W = kl + ku + 1;
  const long long bs = (long long)bp * bp;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) vec[(long long)col_lvl[e] * bp + col_loc[e]] = rhs[e];
  if (e >= (long long)n * W) return;
  const int i = (int)(e / W), t = (int)(e - (long long)i * W);
  const int c = i - kl + t;
  if (c < 0 || c >= n) return;
  const double v = RB[e];
  if (v == 0.0) return;
  const int lr = col_lvl[c], rr = col_loc[c];  // row of G^T
  const int lc = row_lvl[i], rc = row_loc[i];  // column of G^T
  const int kind = lc == lr ? 0 : (lc == lr - 1 ? 1 : 2);
  pool[(long long)(kind * M + lr) * bs + (long long)rr * bp + rc] = v;
}

__global__ void k_bcr_gather_t(const double* __restrict__ xv, const int* __restrict__ row_lvl,
                               const int* __restrict__ row_loc, int n, int bp, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = xv[(long long)row_lvl[i] * bp + row_loc[i]];
}

}  // namespace

size_t adj_smooth_lds_bytes(int m0, int m1, bool f32) {
  const size_t own = 2 * (size_t)m0 * m1 + 2 * (size_t)(m0 + m1);
  return sizeof(double) * ((f32 ? adj_smooth32_off(m0, m1) : smooth_lds_doubles(m0, m1)) + own);
}

size_t adj_basis_lds_bytes(int m0, int m1, int nrhs, bool f32) {
  const size_t own = (size_t)nrhs * m0 * m1;
  return sizeof(double) * ((f32 ? adj_box32_off(m0, m1, nrhs) : box_lds_doubles(m0, m1, nrhs)) + own);
}

size_t adj_part_lds_bytes(int m0, int m1, bool f32) {
  const size_t own = (size_t)m0 * m1 + 2 * (size_t)(m0 + m1);
  return sizeof(double) * ((f32 ? adj_box32_off(m0, m1, 1) : box_lds_doubles(m0, m1, 1) + NBW) + own);
}

template <typename KF>
static hipError_t lds_attr(KF kern, size_t bytes) {
  if (bytes > 64 * 1024)
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return hipSuccess;
}

hipError_t launch_adj_out(const Geo& g, const double* K, const double* p, const double* bcv,
                          const double* dJdp, const double* dJdf, double* meanp, double* pb,
                          double* gfb, double* Kb, hipStream_t s) {
  if (dJdp && g.neumann) hipLaunchKernelGGL(k_adj_mean, dim3(1), dim3(256), 0, s, dJdp, g.ncells, meanp);
  hipLaunchKernelGGL(k_adj_out, dim3((g.ncells + 255) / 256), dim3(256), 0, s, g, K, p, bcv, dJdp,
                     dJdf, meanp, pb, gfb, Kb);
  return hipGetLastError();
}

hipError_t launch_adj_smooth(const Geo& g, const Box* boxes, const int* members, int nmem,
                             const double* K, const double* f, const double* bcv, double beta,
                             const double* fac, const double* fact, const double* tcoup,
                             const Adj32* f32, const double* p_in, const double* gf_in, double* pb,
                             double* gfb, double* Kb, size_t lds, hipStream_t s) {
  if (nmem <= 0) return hipSuccess;
  const Adj32 rf = f32 ? *f32 : Adj32{};
  hipError_t e;
  if (f32) {
    e = lds_attr(k_adj_smooth<true>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_smooth<true>, dim3(nmem), dim3(kAdjNT), lds, s, g, boxes, members, K, f,
                       bcv, beta, fac, fact, tcoup, rf, p_in, gf_in, pb, gfb, Kb);
  } else {
    e = lds_attr(k_adj_smooth<false>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_smooth<false>, dim3(nmem), dim3(kAdjNT), lds, s, g, boxes, members, K, f,
                       bcv, beta, fac, fact, tcoup, rf, p_in, gf_in, pb, gfb, Kb);
  }
  return hipGetLastError();
}

hipError_t launch_adj_combine(const Geo& g, const int* seed_sub, int nX, const double* X,
                              const double* Pk, const double* tr_u, const double* pb,
                              const double* gfb, double* Xb, double* tr_ub, hipStream_t s) {
  if (nX <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_combine, dim3(nX), dim3(256), 0, s, g, seed_sub, X, Pk, tr_u, pb, gfb, Xb,
                     tr_ub);
  return hipGetLastError();
}

hipError_t launch_adj_moments(const Geo& g, const Iface* ifc, int nifc, const Seed* basis,
                              const int* seed_off, const double* X, const double* nu,
                              const double* tr_u, const double* tr_beta, double* tr_ub,
                              double* tr_phib, double* tr_betab, double* ubarb, double* pibarb,
                              hipStream_t s) {
  if (nifc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_moments, dim3(nifc), dim3(64), 0, s, g, ifc, basis, seed_off, X, nu, tr_u,
                     tr_beta, tr_ub, tr_phib, tr_betab, ubarb, pibarb);
  return hipGetLastError();
}

hipError_t launch_adj_basis(const Geo& g, const Box* boxes, int nbox, const Seed* seeds,
                            const double* K, double beta, const double* fac, const double* fact,
                            const Adj32* f32, const double* X, const double* pb, const double* tr_u,
                            const double* tr_ub, const double* tr_phib, const double* tr_betab,
                            double* Kb, size_t lds, hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  const Adj32 rf = f32 ? *f32 : Adj32{};
  hipError_t e;
  if (f32) {
    e = lds_attr(k_adj_basis<true>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_basis<true>, dim3(nbox), dim3(64), lds, s, g, boxes, seeds, K, beta, fac,
                       fact, rf, X, pb, tr_u, tr_ub, tr_phib, tr_betab, Kb);
  } else {
    e = lds_attr(k_adj_basis<false>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_basis<false>, dim3(nbox), dim3(64), lds, s, g, boxes, seeds, K, beta, fac,
                       fact, rf, X, pb, tr_u, tr_ub, tr_phib, tr_betab, Kb);
  }
  return hipGetLastError();
}

hipError_t launch_adj_particular(const Geo& g, const Box* boxes, int nbox, const double* K,
                                 const double* bcv, double beta, const double* fac, const Adj32* f32,
                                 const double* pbar, const double* pb, const double* ubarb,
                                 const double* pibarb, double* Kb, size_t lds, hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  const Adj32 rf = f32 ? *f32 : Adj32{};
  hipError_t e;
  if (f32) {
    e = lds_attr(k_adj_particular<true>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_particular<true>, dim3(nbox), dim3(64), lds, s, g, boxes, K, bcv, beta, fac,
                       rf, pbar, pb, ubarb, pibarb, Kb);
  } else {
    e = lds_attr(k_adj_particular<false>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_particular<false>, dim3(nbox), dim3(64), lds, s, g, boxes, K, bcv, beta, fac,
                       rf, pbar, pb, ubarb, pibarb, Kb);
  }
  return hipGetLastError();
}

hipError_t launch_adj_logk(const double* K, const double* Kb, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_logk, dim3((n + 255) / 256), dim3(256), 0, s, K, Kb, n, out);
  return hipGetLastError();
}

hipError_t launch_bcr_scatter_t(const double* RB, const double* rhs, int n, int kl, int ku,
                                const int* row_lvl, const int* row_loc, const int* col_lvl,
                                const int* col_loc, int M, int bp, double* pool, double* vec,
                                hipStream_t s) {
  const long long tot = std::max<long long>((long long)n * (kl + ku + 1), n);
  hipLaunchKernelGGL(k_bcr_scatter_t, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, RB, rhs, n,
                     kl, ku, row_lvl, row_loc, col_lvl, col_loc, M, bp, pool, vec);
  return hipGetLastError();
}

hipError_t launch_bcr_gather_t(const double* xv, const int* row_lvl, const int* row_loc, int n, int bp,
                               double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bcr_gather_t, dim3((n + 255) / 256), dim3(256), 0, s, xv, row_lvl, row_loc, n, bp,
                     out);
  return hipGetLastError();
}

}  // namespace mrcm
