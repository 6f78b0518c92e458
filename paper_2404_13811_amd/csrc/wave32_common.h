// FP32 solves with FP64 iterative refinement on the one-wavefront-per-box
// 2-D layout, shared by the FP32 local kernels (local_wave32.hip) and the
// FP32 form of the adjoint (adjoint.hip): LDS carve-up of a box with its
// diagonal scaling, the FP32 block-tridiagonal factor of the scaled matrix
// A^ = D^-1/2 A D^-1/2 as explicit block inverses, its sweeps, and the
// refinement loop
//     x = 0;  repeat  r = b - A x (FP64);  x += D^-1/2 solve32(D^-1/2 r)
// until the componentwise backward error max_c |r_c| / (|A| |x| + |b|)_c
// is at most tol.
#pragma once
#include "wave_common.h"

namespace mrcm {
namespace wave {

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

__host__ __device__ inline size_t boxr_bytes(int m0, int m1, int nrhs, int nbrhs, int kc = 1) {
  const size_t nc = (size_t)m0 * m1;
  const size_t d = kx_doubles(kc, m0, m1) + (size_t)(m0 + 2) * (m1 + 2) + 3 * nc + nrhs * nc + nc + nbrhs * nc;
  const size_t f = nrhs * nc + 2 * nc + (size_t)(nrhs < 2 ? 2 : nrhs) * NBW + 4;
  return d * sizeof(double) + f * sizeof(float);
}

__device__ __forceinline__ BoxR carve_r(double* base, const Box& B, int nrhs, int nbrhs, int kc = 1) {
  BoxR r;
  r.b.m0 = B.hi[0] - B.lo[0];
  r.b.m1 = B.hi[1] - B.lo[1];
  const int nc = r.b.m0 * r.b.m1;
  base = attach_kx(r.b, base, kc);
  r.b.Kt = base;
  attach_ky(r.b);
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
  const double kc = kat(R.b, B, x, y, a);
  const double bt = robin_beta(g, a, kc, kat(R.b, B, ox, oy, a), beta);
  const int c[3] = {x, y, 0};
  return robin_T(g, kc, bt) * seed_value(g, sd, B.lo, B.hi, c);
}

// Iterative refinement of nrhs systems A x_k = b_k; b from seeds (if
// seeds != nullptr) or from R.Bv (nrhs x ncell).  Returns the number of
// FP32 solves.
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
        const double bv = seeds ? seed_rhs(g, B, R, seeds[B.seed0 + k], beta, loc) : R.Bv[(size_t)k * nc + loc];
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

// The refinement arrays of a smoothing box, after its carve_smooth layout
// (smooth32_lds_bytes in all).
__device__ __forceinline__ BoxR carve_smooth_r(double* base, const SmoothLds& r) {
  const int nc = r.b.m0 * r.b.m1;
  BoxR R;
  R.b = r.b;
  R.sd = r.b.Z + 2 * NBW;
  R.Bv = R.sd + nc;
  float* fb = reinterpret_cast<float*>(R.Bv + nc);
  R.Wf = fb;
  R.Txf = R.Wf + nc;
  R.Tnf = R.Txf + nc;
  R.Zf = align16(base, R.Tnf + nc);
  return R;
}

__host__ __device__ inline size_t smooth32_lds_bytes(int m0, int m1, int kc = 1) {
  const size_t nc = (size_t)m0 * m1;
  return sizeof(double) * (smooth_lds_doubles(m0, m1, kc) + 2 * nc) + sizeof(float) * (3 * nc + 2 * NBW + 4);
}

}  // namespace wave
}  // namespace mrcm
