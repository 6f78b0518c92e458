// FP32 local factorisations and solves with FP64 iterative refinement, for
// the 2-D boxes handled by the one-wavefront-per-box kernels.
//
// The block-tridiagonal factorisation of local_wave.hip is applied in FP32
// to the symmetrically scaled matrix  A^ = D^-1/2 A D^-1/2  (D = diag A,
// which removes the permeability contrast from the diagonal), and stored
// as FP32 block inverses (half the bytes of the FP64 form).  Every local
// solve is then refined in FP64:
//     x = 0;  repeat  r = b - A x (FP64, two-point stencil from K in LDS);
//                     x += D^-1/2 solve32(D^-1/2 r)
// until the componentwise backward error
//     max_c |r_c| / (|A| |x| + |b|)_c  <=  tol
// or max_refine corrections have been applied (flag MRCM_ENOCONV).  The
// interface system and every reduction stay in FP64.
#include "wave_common.h"

namespace mrcm {
namespace {

using namespace wave;

using WaveSmemF = GjSmem<float>;

// LDS of one box for the refinement kernels.
struct BoxR {
  BoxLds b;     // Kt, Dg, Tx, Tn (FP64); b.X = solution x (nrhs x ncell)
  double* sd;   // ncell, 1 / sqrt(diag)
  double* Bv;   // nb_rhs x ncell right-hand sides (not stored for seeds)
  float* Wf;    // nrhs x ncell FP32 work vectors
  float* Txf;   // ncell scaled x couplings
  float* Tnf;   // ncell scaled block couplings
  float* Zf;    // nrhs x NBW staging
};

__host__ __device__ inline size_t boxr_bytes(int m0, int m1, int nrhs, int nbrhs) {
  const size_t nc = (size_t)m0 * m1;
  const size_t d = (size_t)(m0 + 2) * (m1 + 2) + 3 * nc + nrhs * nc + nc + nbrhs * nc;
  const size_t f = nrhs * nc + 2 * nc + (size_t)(nrhs < 2 ? 2 : nrhs) * NBW + 4;
  return d * sizeof(double) + f * sizeof(float);
}

__device__ __forceinline__ BoxR carve_r(double* base, const Box& B, int nrhs, int nbrhs) {
  BoxR r;
  r.b.m0 = B.hi[0] - B.lo[0];
  r.b.m1 = B.hi[1] - B.lo[1];
  const int nc = r.b.m0 * r.b.m1;
  r.b.Kt = base;
  r.b.Dg = r.b.Kt + (r.b.m0 + 2) * (r.b.m1 + 2);
  r.b.Tx = r.b.Dg + nc;
  r.b.Tn = r.b.Tx + nc;
  r.b.X = r.b.Tn + nc;
  r.sd = r.b.X + (size_t)nrhs * nc;
  r.Bv = r.sd + nc;
  r.b.Z = nullptr;
  float* fb = reinterpret_cast<float*>(r.Bv + (size_t)nbrhs * nc);
  r.Wf = fb;
  r.Txf = r.Wf + (size_t)nrhs * nc;
  r.Tnf = r.Txf + nc;
  r.Zf = align16(base, r.Tnf + nc);
  return r;
}

// Scale factors and scaled couplings (after load_box).
template <int NT = 64>
__device__ __forceinline__ void scale_box(const Box& B, BoxR& R) {
  const int nc = B.ncell, nb = B.nb;
  const int tid = threadIdx.x % NT;
#pragma unroll 1
  for (int e = tid; e < nc; e += NT) R.sd[e] = rcp_d(sqrt(R.b.Dg[e]));
  bsync<NT>();
#pragma unroll 1
  for (int e = tid; e < nc; e += NT) {
    const int xl = e % R.b.m0;
    R.Txf[e] = (xl + 1 < R.b.m0) ? (float)(R.b.Tx[e] * R.sd[e] * R.sd[e + 1]) : 0.0f;
    R.Tnf[e] = (e + nb < nc) ? (float)(R.b.Tn[e] * R.sd[e] * R.sd[e + nb]) : 0.0f;
  }
  bsync<NT>();
}


// Scaled S_j into w (column c, my half), w = W_{j-1} on entry when j > 0
// (branch-free, as wbuild).
__device__ __forceinline__ void wbuild32(int nb, int j, const BoxR& R, float w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int cc = c < nb ? c : 0;
  const float* Tx = R.Txf + j * nb;
  const float* Tp = R.Tnf + (j - 1) * nb;  // read only when j > 0
  const float txc = Tx[cc];
  const float tc = j > 0 ? Tp[cc] : 0.0f;
  float tr[HB], tpr[HB];
#pragma unroll
  for (int i = 0; i < HB; ++i) {
    const int r = HB * h + i;
    const int rr = r < nb ? r : 0;
    tr[i] = Tx[rr];
    tpr[i] = j > 0 ? Tp[rr] : 0.0f;
  }
#pragma unroll
  for (int i = 0; i < HB; ++i) {
    const int r = HB * h + i;
    const int d = r - c;
    float v = d == 0 ? 1.0f : d == -1 ? -tr[i] : d == 1 ? -txc : 0.0f;
    v = fmaf(-tpr[i] * tc, w[i], v);
    w[i] = (r < nb && c < nb) ? v : (d == 0 ? 1.0f : 0.0f);
  }
}

__device__ __forceinline__ void wgj32(int nb, WaveSmemF& sm, float w[HB]) { wgj_blk<float>(nb, sm, w); }

// W_j z with 128-bit LDS reads, two FMA chains and the half-wave swap sum.
__device__ __forceinline__ float wgemv2f(const float w[HB], const float* z) {
  const int h = lane_id() >> 5;
  const float4* z4 = reinterpret_cast<const float4*>(z + HB * h);
  float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
  for (int i = 0; i < HB / 4; ++i) {
    const float4 v = z4[i];
    a0 = fmaf(w[4 * i], v.x, a0);
    a1 = fmaf(w[4 * i + 1], v.y, a1);
    a0 = fmaf(w[4 * i + 2], v.z, a0);
    a1 = fmaf(w[4 * i + 3], v.w, a1);
  }
  return half_sum_f(a0 + a1);
}



__device__ __forceinline__ void fwd32(int nb, int nc, int j, int nrhs, const BoxR& R, const float w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  #pragma unroll 1
  for (int e = L; e < nrhs * NBW; e += 64) {
    const int k = e / NBW, r = e % NBW;
    float v = 0.0f;
    if (r < nb) {
      v = R.Wf[k * nc + j * nb + r];
      if (j > 0) v += R.Tnf[(j - 1) * nb + r] * R.Wf[k * nc + (j - 1) * nb + r];
    }
    R.Zf[k * NBW + r] = v;
  }
  wsync();
  for (int k = 0; k < nrhs; ++k) {
    const float y = wgemv2f(w, R.Zf + k * NBW);
    if (h == 0 && c < nb) R.Wf[k * nc + j * nb + c] = y;
  }
  wsync();
}

__device__ __forceinline__ void bwd32(int nb, int nc, int j, int nrhs, const BoxR& R, const float w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  #pragma unroll 1
  for (int e = L; e < nrhs * NBW; e += 64) {
    const int k = e / NBW, r = e % NBW;
    R.Zf[k * NBW + r] = (r < nb) ? R.Tnf[j * nb + r] * R.Wf[k * nc + (j + 1) * nb + r] : 0.0f;
  }
  wsync();
  for (int k = 0; k < nrhs; ++k) {
    const float y = wgemv2f(w, R.Zf + k * NBW);
    if (h == 0 && c < nb) R.Wf[k * nc + j * nb + c] += y;
  }
  wsync();
}

__device__ __forceinline__ void factor32(const Box& B, float* Wg, const BoxR& R, WaveSmemF& sm) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb;
  float w[HB];
#pragma unroll
  for (int i = 0; i < HB; ++i) w[i] = 0.0f;
  for (int j = 0; j < B.nblk; ++j) {
    wbuild32(nb, j, R, w);
    wgj32(nb, sm, w);
    float* Wj = Wg + (long long)j * nb * nb;
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const int r = HB * h + i;
      if (r < nb && c < nb) Wj[r * nb + c] = w[i];
    }
  }
  wsync();
}

// FP32 solve of the scaled system on every work vector in R.Wf.
__device__ __forceinline__ void solve32(const Box& B, const float* Wg, int nrhs, const BoxR& R) {
  const int nb = B.nb, nblk = B.nblk, nc = B.ncell;
  const long long bs = (long long)nb * nb;
  const BlockSrc<float> src = block_src(Wg, nb, nblk);
  {
    float w[RING][HB];
#pragma unroll
    for (int q = 0; q < RING; ++q)
      if (q < nblk) wload_block(src, q, w[q]);
    for (int j0 = 0; j0 < nblk; j0 += RING) {
#pragma unroll
      for (int q = 0; q < RING; ++q) {
        const int j = j0 + q;
        if (j < nblk) {
          fwd32(nb, nc, j, nrhs, R, w[q]);
          if (j + RING < nblk) wload_block(src, (j + RING), w[q]);
        }
      }
    }
  }
  {
    float w[RING][HB];
#pragma unroll
    for (int q = 0; q < RING; ++q)
      if (nblk - 2 - q >= 0) wload_block(src, (nblk - 2 - q), w[q]);
    for (int t0 = 0; t0 <= nblk - 2; t0 += RING) {
#pragma unroll
      for (int q = 0; q < RING; ++q) {
        const int j = nblk - 2 - (t0 + q);
        if (j >= 0) {
          bwd32(nb, nc, j, nrhs, R, w[q]);
          if (j - RING >= 0) wload_block(src, (j - RING), w[q]);
        }
      }
    }
  }
}

// Single right-hand side in R.Wf: forward and backward sweeps with the
// previous block's values kept in registers (as the FP64 sweep).
__device__ __forceinline__ void sweep1f(const Box& B, const float* Wg, const BoxR& R) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb, nblk = B.nblk;
  const bool cv = c < nb;
  const long long bs = (long long)nb * nb;
  const BlockSrc<float> src = block_src(Wg, nb, nblk);
  float* X = R.Wf;
  const float* Tn = R.Tnf;
  float* z = R.Zf;
  {
    float w[RING][HB];
#pragma unroll
    for (int q = 0; q < RING; ++q)
      if (q < nblk) wload_block(src, q, w[q]);
    float y = 0.0f, xn = cv ? X[c] : 0.0f, tp = 0.0f;
    for (int j0 = 0; j0 < nblk; j0 += RING) {
#pragma unroll
      for (int q = 0; q < RING; ++q) {
        const int j = j0 + q;
        if (j < nblk) {
          float* zb = z + (j & 1) * NBW;
          if (h == 0) zb[c] = cv ? fmaf(tp, y, xn) : 0.0f;
          __builtin_amdgcn_wave_barrier();
          const bool more = j + 1 < nblk;
          xn = (more && cv) ? X[(j + 1) * nb + c] : 0.0f;
          tp = (more && cv) ? Tn[j * nb + c] : 0.0f;
          y = wgemv2f(w[q], zb);
          if (h == 0 && cv) X[j * nb + c] = y;
          if (j + RING < nblk) wload_block(src, (j + RING), w[q]);
        }
      }
    }
  }
  {
    float w[RING][HB];
#pragma unroll
    for (int q = 0; q < RING; ++q)
      if (nblk - 2 - q >= 0) wload_block(src, (nblk - 2 - q), w[q]);
    __builtin_amdgcn_wave_barrier();
    float xnext = cv ? X[(nblk - 1) * nb + c] : 0.0f;
    float tj = (nblk >= 2 && cv) ? Tn[(nblk - 2) * nb + c] : 0.0f;
    float wj = (nblk >= 2 && cv) ? X[(nblk - 2) * nb + c] : 0.0f;
    for (int t0 = 0; t0 <= nblk - 2; t0 += RING) {
#pragma unroll
      for (int q = 0; q < RING; ++q) {
        const int j = nblk - 2 - (t0 + q);
        if (j >= 0) {
          float* zb = z + (j & 1) * NBW;
          if (h == 0) zb[c] = cv ? tj * xnext : 0.0f;
          __builtin_amdgcn_wave_barrier();
          const float wcur = wj;
          tj = (j >= 1 && cv) ? Tn[(j - 1) * nb + c] : 0.0f;
          wj = (j >= 1 && cv) ? X[(j - 1) * nb + c] : 0.0f;
          xnext = wcur + wgemv2f(w[q], zb);
          if (h == 0 && cv) X[j * nb + c] = xnext;
          if (j - RING >= 0) wload_block(src, (j - RING), w[q]);
        }
      }
    }
  }
  wsync();
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Maximum over the wave of non-negative values: quad and row steps by DPP,
// then the row pairs and the half-waves by lane swaps (no LDS).
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<0xB1>(v));   // quad_perm(1,0,3,2)
  v = fmax(v, dpp_d<0x4E>(v));   // quad_perm(2,3,0,1)
  v = fmax(v, dpp_d<0x124>(v));  // row_ror:4
  v = fmax(v, dpp_d<0x128>(v));  // row_ror:8
  {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const auto l2 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h2 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    v = fmax(__hiloint2double(h2[0], l2[0]), __hiloint2double(h2[1], l2[1]));
  }
  {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const auto l2 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h2 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    v = fmax(__hiloint2double(h2[0], l2[0]), __hiloint2double(h2[1], l2[1]));
  }
  return v;
}

// Right-hand side of seed k at box cell loc (T^R times the seed on its side).
__device__ __forceinline__ double seed_rhs(const Geo& g, const Box& B, const BoxR& R, const Seed& sd,
                                           double beta, int loc) {
  const int x = B.lo[0] + loc % R.b.m0, y = B.lo[1] + loc / R.b.m0;
  const int a = sd.side >> 1, so = sd.side & 1;
  const bool on = (a == 0) ? (x == (so ? B.hi[0] - 1 : B.lo[0])) : (y == (so ? B.hi[1] - 1 : B.lo[1]));
  if (!on) return 0.0;
  const int ox = x + (a == 0 ? (so ? 1 : -1) : 0), oy = y + (a == 1 ? (so ? 1 : -1) : 0);
  const double kc = kat(R.b, B, x, y);
  const double bt = robin_beta(g, a, kc, kat(R.b, B, ox, oy), beta);
  const int c[3] = {x, y, 0};
  return robin_T(g, kc, bt) * seed_value(g, sd, B.lo, B.hi, c);
}

// Iterative refinement of nrhs systems A x_k = b_k; b from seeds (if
// seeds != nullptr) or from R.Bv.  Returns the number of FP32 solves.
template <bool ONE>
__device__ __forceinline__ int refine(const Geo& g, const Box& B, const BoxR& R, const float* Wg, int nrhs,
                      const Seed* seeds, double beta, double tol, int max_refine, double& omega_out,
                      WaveSmemF& sm) {
  const int L = lane_id();
  const int nc = B.ncell, m0 = R.b.m0, nb = B.nb;
  for (int e = L; e < nrhs * nc; e += 64) R.b.X[e] = 0.0;
  wsync();
  int it = 0;
  double omega = 0.0;
  while (true) {
    // r = b - A x, scaled into the FP32 work vectors; componentwise backward error
    omega = 0.0;
    for (int k = 0; k < nrhs; ++k) {
      const double* x = R.b.X + (size_t)k * nc;
      double om = 0.0;
      #pragma unroll 1
      for (int loc = L; loc < nc; loc += 64) {
        const double bv = seeds ? seed_rhs(g, B, R, seeds[B.seed0 + k], beta, loc) : R.Bv[loc];
        const int xl = loc % m0;
        const double xc = x[loc];
        double ax = R.b.Dg[loc] * xc, aa = fabs(R.b.Dg[loc] * xc);
        if (xl > 0) { const double t = R.b.Tx[loc - 1] * x[loc - 1]; ax -= t; aa += fabs(t); }
        if (xl + 1 < m0) { const double t = R.b.Tx[loc] * x[loc + 1]; ax -= t; aa += fabs(t); }
        if (loc >= nb) { const double t = R.b.Tn[loc - nb] * x[loc - nb]; ax -= t; aa += fabs(t); }
        if (loc + nb < nc) { const double t = R.b.Tn[loc] * x[loc + nb]; ax -= t; aa += fabs(t); }
        const double r = bv - ax;
        const double den = aa + fabs(bv);
        // a non-finite residual or iterate never counts as converged (fmax
        // would drop a NaN ratio)
        if (!(r - r == 0.0 && den - den == 0.0)) om = INFINITY;
        else if (den > 0.0) om = fmax(om, fabs(r) / den);
        R.Wf[(size_t)k * nc + loc] = (float)(R.sd[loc] * r);
      }
      omega = fmax(omega, wave_max(om));
    }
    wsync();
    if (it > 0 && omega <= tol) break;
    if (it > max_refine || !(omega <= 1e300)) {
      if (L == 0) sm.flag |= kFlagNoConv;
      break;
    }
    if (ONE) sweep1f(B, Wg, R);
    else solve32(B, Wg, nrhs, R);
    for (int e = L; e < nrhs * nc; e += 64) R.b.X[e] += R.sd[e % nc] * (double)R.Wf[e];
    wsync();
    ++it;
  }
  omega_out = omega;
  return it;
}

__device__ __forceinline__ void record_refine(int it, double omega, int* iters,
                                              unsigned long long* resid) {
  if (lane_id() == 0) {
    atomicMax(iters, it);
    atomicMax(resid, (unsigned long long)__double_as_longlong(omega));
  }
}

// ------------------------------------------------------------------ kernels

// Steps 1-2 on an oversampled box: FP32 factor, seeds refined to tol.
__device__ __forceinline__ void basis32_box(const Geo& g, const Box& B, const Seed* __restrict__ seeds,
                                            const double* __restrict__ K, double beta,
                                            float* __restrict__ fac32, double* __restrict__ Pk,
                                            double* __restrict__ tr_u, double* __restrict__ tr_phi,
                                            double* __restrict__ tr_beta, double tol, int max_refine,
                                            int* iters, unsigned long long* resid, double* dsm,
                                            WaveSmemF& sm) {
  const int L = lane_id();
  const int nrhs = B.nrhs;
  BoxR R = carve_r(dsm, B, max(nrhs, 1), 0);
  load_box(g, B, K, beta, R.b);
  scale_box(B, R);
  float* Wg = fac32 + B.fac;
  factor32(B, Wg, R, sm);
  double omega = 0.0;
  const int it = nrhs > 0 ? refine<false>(g, B, R, Wg, nrhs, seeds, beta, tol, max_refine, omega, sm) : 0;
  record_refine(it, omega, iters, resid);
  const BoxLds& s = R.b;
  const int nc = B.ncell;
  int olo[3], ohi[3];
  womega(g, B.sub, olo, ohi);
  const int ncell_o = g.S[0] * g.S[1];
  #pragma unroll 1
  for (int e = L; e < nrhs * ncell_o; e += 64) {
    const int k = e / ncell_o, t = e % ncell_o;
    Pk[(long long)(B.seed0 + k) * ncell_o + t] =
        s.X[k * nc + bloc(B, s, olo[0] + t % g.S[0], olo[1] + t / g.S[0])];
  }
  for (int q = 0; q < 4; ++q) {
    const int nf = (q >> 1) == 0 ? g.S[1] : g.S[0];
    const bool has = wneighbor(g, B.sub, q) >= 0;
    const int a = q >> 1, so = q & 1;
    #pragma unroll 1
    for (int e = L; e < nrhs * nf; e += 64) {
      const int k = e / nf, t = e % nf;
      const long long oidx = (long long)(B.seed0 + k) * g.gstride + g.gside_off[q] + t;
      if (!has) {
        tr_u[oidx] = 0.0;
        tr_phi[oidx] = 0.0;
        continue;
      }
      int x, y;
      wgface(olo, ohi, q, t, x, y);
      const int ox = x + (a == 0 ? (so ? 1 : -1) : 0), oy = y + (a == 1 ? (so ? 1 : -1) : 0);
      const double kc = kat(s, B, x, y), ko = kat(s, B, ox, oy);
      const double Pc = s.X[k * nc + bloc(B, s, x, y)];
      const double bt = robin_beta(g, a, kc, ko, beta);
      double u;
      if (win_box(B, ox, oy)) {
        u = g.area * kharm(kc, ko) / g.h * (Pc - s.X[k * nc + bloc(B, s, ox, oy)]) / g.area;
      } else {
        const Seed sd = seeds[B.seed0 + k];
        const int c[3] = {x, y, 0};
        const double lam = (sd.side == q) ? seed_value(g, sd, B.lo, B.hi, c) : 0.0;
        u = robin_T(g, kc, bt) * (Pc - lam) / g.area;
      }
      const double pi = Pc - u * g.h / (2.0 * kc);
      tr_u[oidx] = u;
      tr_phi[oidx] = -bt * u + pi;
      if (k == 0) tr_beta[(long long)B.sub * g.gstride + g.gside_off[q] + t] = bt;
    }
  }
}

// Step 4 on a subdomain: FP32 factor, particular solution refined to tol.
__device__ __forceinline__ void particular32_box(const Geo& g, const Box& B, const double* __restrict__ K,
                                                 const double* __restrict__ f,
                                                 const double* __restrict__ bcv, double beta,
                                                 float* __restrict__ fac32, double* __restrict__ pbar,
                                                 double* __restrict__ ubar, double* __restrict__ pibar,
                                                 double tol, int max_refine, int* iters,
                                                 unsigned long long* resid, double* dsm,
                                                 WaveSmemF& sm) {
  const int L = lane_id();
  BoxR R = carve_r(dsm, B, 1, 1);
  load_box(g, B, K, beta, R.b);
  scale_box(B, R);
  physical_rhs(g, B, R.b, f, bcv, R.Bv);
  wsync();
  float* Wg = fac32 + B.fac;
  factor32(B, Wg, R, sm);
  double omega = 0.0;
  const int it = refine<true>(g, B, R, Wg, 1, nullptr, beta, tol, max_refine, omega, sm);
  record_refine(it, omega, iters, resid);
  const BoxLds& s = R.b;
  for (int t = L; t < B.ncell; t += 64) pbar[(long long)B.sub * B.ncell + t] = s.X[t];
  for (int q = 0; q < 4; ++q) {
    const int nf = (q >> 1) == 0 ? g.S[1] : g.S[0];
    const bool has = wneighbor(g, B.sub, q) >= 0;
    const int a = q >> 1, so = q & 1;
    #pragma unroll 1
    for (int t = L; t < nf; t += 64) {
      const long long oidx = (long long)B.sub * g.gstride + g.gside_off[q] + t;
      if (!has) {
        ubar[oidx] = 0.0;
        pibar[oidx] = 0.0;
        continue;
      }
      int x, y;
      wgface(B.lo, B.hi, q, t, x, y);
      const int ox = x + (a == 0 ? (so ? 1 : -1) : 0), oy = y + (a == 1 ? (so ? 1 : -1) : 0);
      const double kc = kat(s, B, x, y);
      const double bt = robin_beta(g, a, kc, kat(s, B, ox, oy), beta);
      const double u = robin_T(g, kc, bt) * s.X[bloc(B, s, x, y)] / g.area;
      ubar[oidx] = u;
      pibar[oidx] = bt * u;
    }
  }
}

// Steps 1-2 and 4 in one launch: workgroups [0, nbox) take the oversampled
// boxes, workgroups [nbox, 2 nbox) the particular problems.  The two sets are
// independent and run side by side.
__global__ void __launch_bounds__(64) k_local32(Geo g, const Box* __restrict__ obox,
                                                const Box* __restrict__ pbox, int nbox,
                                                const Seed* __restrict__ seeds,
                                                const double* __restrict__ K,
                                                const double* __restrict__ f,
                                                const double* __restrict__ bcv, double beta,
                                                float* __restrict__ fac32,
                                                float* __restrict__ facp32,
                                                double* __restrict__ Pk,
                                                double* __restrict__ tr_u,
                                                double* __restrict__ tr_phi,
                                                double* __restrict__ tr_beta,
                                                double* __restrict__ pbar,
                                                double* __restrict__ ubar,
                                                double* __restrict__ pibar, double tol,
                                                int max_refine, int* iters,
                                                unsigned long long* resid, int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ WaveSmemF sm;
  const int L = lane_id();
  if (L == 0) sm.flag = 0;
  const int b = blockIdx.x;
  if (b < nbox) {
    const Box B = obox[b];
    basis32_box(g, B, seeds, K, beta, fac32, Pk, tr_u, tr_phi, tr_beta, tol, max_refine, iters,
                resid, dsm, sm);
  } else {
    const Box B = pbox[b - nbox];
    particular32_box(g, B, K, f, bcv, beta, facp32, pbar, ubar, pibar, tol, max_refine, iters,
                     resid, dsm, sm);
  }
  wsync();
  if (L == 0 && sm.flag) atomicOr(flags, sm.flag);
}

// Algorithm 1, Step 6 in the FP32 form: the oversampled boxes factored
// again (FP32, diagonally scaled) with the smoothing Robin parameter; no
// right-hand side is solved.
__global__ void __launch_bounds__(64) k_factor32(Geo g, const Box* __restrict__ obox,
                                                 const double* __restrict__ K, double beta,
                                                 float* __restrict__ fac32, int* iters,
                                                 unsigned long long* resid, int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ WaveSmemF sm;
  const int L = lane_id();
  if (L == 0) sm.flag = 0;
  Box B = obox[blockIdx.x];
  B.nrhs = 0;
  basis32_box(g, B, nullptr, K, beta, fac32, nullptr, nullptr, nullptr, nullptr, 1.0, 0, iters,
              resid, dsm, sm);
  wsync();
  if (L == 0 && sm.flag) atomicOr(flags, sm.flag);
}

__host__ __device__ inline size_t smooth32_lds_bytes(int m0, int m1) {
  const size_t nc = (size_t)m0 * m1;
  return sizeof(double) * (smooth_lds_doubles(m0, m1) + 2 * nc) + sizeof(float) * (3 * nc + 2 * NBW + 4);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_smooth32(Geo g, const Box* __restrict__ boxes,
                                                 const double* __restrict__ K,
                                                 const double* __restrict__ f,
                                                 const double* __restrict__ bcv, double beta,
                                                 const float* __restrict__ fac32,
                                                 double* __restrict__ p,
                                                 double* __restrict__ gflux, double tol,
                                                 int max_refine, int* iters,
                                                 unsigned long long* resid, int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ WaveSmemF sm;
  const Box B = boxes[blockIdx.x];
  if (threadIdx.x == 0) sm.flag = 0;
  SmoothLds r = carve_smooth(dsm, B);
  const int nc = B.ncell;
  BoxR R;
  R.b = r.b;
  R.sd = r.b.Z + 2 * NBW;
  R.Bv = R.sd + nc;
  float* fb = reinterpret_cast<float*>(R.Bv + nc);
  R.Wf = fb;
  R.Txf = R.Wf + nc;
  R.Tnf = R.Txf + nc;
  R.Zf = align16(dsm, R.Tnf + nc);
  stage_smooth<NT>(g, B, r, K, p, f, gflux, bcv, nullptr);
  __syncthreads();
  smooth_rhs<NT>(g, B, r, beta, R.Bv);
  coef_box<NT>(g, B, beta, R.b);
  scale_box<NT>(B, R);
  if (threadIdx.x < 64) {
    double omega = 0.0;
    const int it = refine<true>(g, B, R, fac32 + B.fac, 1, nullptr, beta, tol, max_refine, omega, sm);
    record_refine(it, omega, iters, resid);
  }
  __syncthreads();
  smooth_out<NT>(g, B, r, R.b.X, beta, p, gflux);
  if (threadIdx.x == 0 && sm.flag) atomicOr(flags, sm.flag);
}

template <typename KF>
hipError_t set_lds(KF kern, size_t bytes) {
  if (bytes > 64 * 1024)
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
  return hipSuccess;
}

}  // namespace

size_t wave32_lds_bytes(int m0, int m1, int nrhs, int nbrhs) { return boxr_bytes(m0, m1, nrhs, nbrhs); }

size_t wave32_smooth_lds_bytes(int m0, int m1) { return smooth32_lds_bytes(m0, m1); }

hipError_t launch_local32_w(const Geo& g, const Box* obox, const Box* pbox, int nbox,
                            const Seed* seeds, const double* K, const double* f, const double* bcv,
                            double beta, float* fac32, float* facp32, double* Pk, double* tr_u,
                            double* tr_phi, double* tr_beta, double* pbar, double* ubar,
                            double* pibar, double tol, int max_refine, int* iters,
                            unsigned long long* resid, int* flags, size_t lds, hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  hipError_t e = set_lds(k_local32, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_local32, dim3(2 * nbox), dim3(64), lds, s, g, obox, pbox, nbox, seeds, K, f,
                     bcv, beta, fac32, facp32, Pk, tr_u, tr_phi, tr_beta, pbar, ubar, pibar, tol,
                     max_refine, iters, resid, flags);
  return hipGetLastError();
}

hipError_t launch_factor32_w(const Geo& g, const Box* obox, int nbox, const double* K, double beta,
                             float* fac32, int* iters, unsigned long long* resid, int* flags,
                             size_t lds, hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  hipError_t e = set_lds(k_factor32, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_factor32, dim3(nbox), dim3(64), lds, s, g, obox, K, beta, fac32, iters,
                     resid, flags);
  return hipGetLastError();
}

hipError_t launch_smooth32_w(const Geo& g, const Box* boxes, int nmem,
                             const double* K, const double* f, const double* bcv, double beta,
                             const float* fac32, double* p, double* gflux, double tol,
                             int max_refine, int* iters, unsigned long long* resid, int* flags,
                             size_t lds, int nt, hipStream_t s) {
  if (nmem <= 0) return hipSuccess;
  hipError_t e;
#define MRCM_SMOOTH32_NT(N)                                                                     \
  e = set_lds(k_smooth32<N>, lds);                                                              \
  if (e != hipSuccess) return e;                                                                \
  hipLaunchKernelGGL(k_smooth32<N>, dim3(nmem), dim3(N), lds, s, g, boxes, K, f, bcv,           \
                     beta, fac32, p, gflux, tol, max_refine, iters, resid, flags);
  if (nt == 64) {
    MRCM_SMOOTH32_NT(64)
  } else if (nt == 128) {
    MRCM_SMOOTH32_NT(128)
  } else if (nt == 256) {
    MRCM_SMOOTH32_NT(256)
  } else {
    return hipErrorInvalidValue;
  }
#undef MRCM_SMOOTH32_NT
  return hipGetLastError();
}

}  // namespace mrcm
