// One-wavefront-per-box kernels for the 2-D local problems (dense blocks of
// at most 32 cells): factorisation with the seed solves fused into its
// forward sweep, particular problems, and one color phase of smoothing.
//
// Register layout of a 32 x 32 block (padded with the identity when the box
// line is shorter): lane L holds rows 16h .. 16h+15 of column c, with
// c = L & 31 and h = L >> 5, so all 64 lanes carry work.
//
// The block inverse is computed by in-place Gauss-Jordan elimination (no
// pivoting: the pivots of an SPD matrix are positive).  Each step broadcasts
// pivot row and column through LDS; no cross-lane reduction and no barrier
// beyond the single wave.
//
// Solves use the block LDL^T recurrences of the block-tridiagonal matrix
// (see local.hip): forward w_j = W_j (b_j + t_{j-1} .* w_{j-1}), backward
// x_j = w_j + W_j (t_j .* x_{j+1}).  A block product is a 16-term dot
// product per lane followed by one exchange between the two half-waves.
//
// Everything a sweep touches between block steps lives in LDS: the box's
// permeabilities (with a one-cell halo), its diagonal and couplings, and
// the right-hand sides / solutions.  The cached block inverses are streamed
// from memory four blocks ahead of their use.
#include "wave_common.h"

namespace mrcm {
namespace {

using namespace wave;



// W_j z for the block staged in z (LDS): lane (c, h) sums its 16 rows with
// two accumulators; half_sum completes the column.
__device__ __forceinline__ double wgemv2(const double w[HB], const double* z) {
  const int h = lane_id() >> 5;
  const double2* z2 = reinterpret_cast<const double2*>(z + HB * h);
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int i = 0; i < HB / 2; ++i) {
    const double2 v = z2[i];
    a0 = fma(w[2 * i], v.x, a0);
    a1 = fma(w[2 * i + 1], v.y, a1);
  }
  return half_sum(a0 + a1);
}

// Forward step of block j for all right-hand sides, inverse in w:
// X_j <- W_j (X_j + t_{j-1} .* X_{j-1}).
__device__ __forceinline__ void fwd_step(int nb, int ncell, int j, int nrhs, const BoxLds& s,
                                         const double w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  #pragma unroll 1
  for (int e = L; e < nrhs * NBW; e += 64) {
    const int k = e / NBW, r = e % NBW;
    double v = 0.0;
    if (r < nb) {
      v = s.X[k * ncell + j * nb + r];
      if (j > 0) v += s.Tn[(j - 1) * nb + r] * s.X[k * ncell + (j - 1) * nb + r];
    }
    s.Z[k * NBW + r] = v;
  }
  wsync();
  for (int k = 0; k < nrhs; ++k) {
    const double y = wgemv2(w, s.Z + k * NBW);
    if (h == 0 && c < nb) s.X[k * ncell + j * nb + c] = y;
  }
  wsync();
}

// Backward step of block j: X_j <- X_j + W_j (t_j .* X_{j+1}).
__device__ __forceinline__ void bwd_step(int nb, int ncell, int j, int nrhs, const BoxLds& s,
                                         const double w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  #pragma unroll 1
  for (int e = L; e < nrhs * NBW; e += 64) {
    const int k = e / NBW, r = e % NBW;
    s.Z[k * NBW + r] = (r < nb) ? s.Tn[j * nb + r] * s.X[k * ncell + (j + 1) * nb + r] : 0.0;
  }
  wsync();
  for (int k = 0; k < nrhs; ++k) {
    const double y = wgemv2(w, s.Z + k * NBW);
    if (h == 0 && c < nb) s.X[k * ncell + j * nb + c] += y;
  }
  wsync();
}

// Factorisation fused with the forward sweep; inverses to Wg, couplings to Tg.
__device__ __forceinline__ void factor_forward(const Box& B, double* Wg, double* Tg, int nrhs, const BoxLds& s,
                               WaveSmem& sm) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb;
  for (int e = L; e < B.ncell; e += 64) Tg[e] = s.Tn[e];
  double w[HB];
#pragma unroll
  for (int i = 0; i < HB; ++i) w[i] = 0.0;
  for (int j = 0; j < B.nblk; ++j) {
    wbuild(nb, j, s, w);
    wgj(nb, sm, w);
    double* Wj = Wg + (long long)j * nb * nb;
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const int r = HB * h + i;
      if (r < nb && c < nb) Wj[r * nb + c] = w[i];
    }
    fwd_step(nb, B.ncell, j, nrhs, s, w);
  }
}

// Sweeps with the cached inverses streamed from memory, RING blocks ahead.
__device__ __forceinline__ void forward_cached(const Box& B, const double* Wg, int nrhs, const BoxLds& s) {
  const int nb = B.nb, nblk = B.nblk;
  const long long bs = (long long)nb * nb;
  const BlockSrc<double> src = block_src(Wg, nb, nblk);
  double w[RING][HB];
#pragma unroll
  for (int q = 0; q < RING; ++q)
    if (q < nblk) wload_block(src, q, w[q]);
  for (int j0 = 0; j0 < nblk; j0 += RING) {
#pragma unroll
    for (int q = 0; q < RING; ++q) {
      const int j = j0 + q;
      if (j < nblk) {
        fwd_step(nb, B.ncell, j, nrhs, s, w[q]);
        if (j + RING < nblk) wload_block(src, (j + RING), w[q]);
      }
    }
  }
}

__device__ __forceinline__ void backward_cached(const Box& B, const double* Wg, int nrhs, const BoxLds& s) {
  const int nb = B.nb, nblk = B.nblk;
  const long long bs = (long long)nb * nb;
  const BlockSrc<double> src = block_src(Wg, nb, nblk);
  double w[RING][HB];
  // block j = nblk - 2 - t uses ring slot t % RING
#pragma unroll
  for (int q = 0; q < RING; ++q)
    if (nblk - 2 - q >= 0) wload_block(src, (nblk - 2 - q), w[q]);
  for (int t0 = 0; t0 <= nblk - 2; t0 += RING) {
#pragma unroll
    for (int q = 0; q < RING; ++q) {
      const int j = nblk - 2 - (t0 + q);
      if (j >= 0) {
        bwd_step(nb, B.ncell, j, nrhs, s, w[q]);
        if (j - RING >= 0) wload_block(src, (j - RING), w[q]);
      }
    }
  }
}

// Forward and backward sweeps of one right-hand side in s.X with the cached
// inverses.  The value of the previous block stays in registers (every lane
// of column c holds it), so a block step is one LDS write of the staged
// vector, the 16-term products and one half-wave exchange.  z points to
// 2 x NBW doubles of LDS (alternating buffers).
__device__ __forceinline__ void sweep1(const Box& B, const double* Wg, const BoxLds& s, double* z) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb, nblk = B.nblk;
  const bool cv = c < nb;
  const long long bs = (long long)nb * nb;
  const BlockSrc<double> src = block_src(Wg, nb, nblk);
  {
    double w[RING][HB];
#pragma unroll
    for (int q = 0; q < RING; ++q)
      if (q < nblk) wload_block(src, q, w[q]);
    double y = 0.0;
    double xn = cv ? s.X[c] : 0.0, tp = 0.0;
    for (int j0 = 0; j0 < nblk; j0 += RING) {
#pragma unroll
      for (int q = 0; q < RING; ++q) {
        const int j = j0 + q;
        if (j < nblk) {
          double* zb = z + (j & 1) * NBW;
          if (h == 0) zb[c] = cv ? fma(tp, y, xn) : 0.0;
          __builtin_amdgcn_wave_barrier();
          const bool more = j + 1 < nblk;
          xn = (more && cv) ? s.X[(j + 1) * nb + c] : 0.0;
          tp = (more && cv) ? s.Tn[j * nb + c] : 0.0;
          y = wgemv2(w[q], zb);
          if (h == 0 && cv) s.X[j * nb + c] = y;
          if (j + RING < nblk) wload_block(src, (j + RING), w[q]);
        }
      }
    }
  }
  {
    double w[RING][HB];
#pragma unroll
    for (int q = 0; q < RING; ++q)
      if (nblk - 2 - q >= 0) wload_block(src, (nblk - 2 - q), w[q]);
    // x_{nblk-1} = w_{nblk-1} is final; every lane of column c reads it
    __builtin_amdgcn_wave_barrier();
    double xnext = cv ? s.X[(nblk - 1) * nb + c] : 0.0;
    double tj = (nblk >= 2 && cv) ? s.Tn[(nblk - 2) * nb + c] : 0.0;
    double wj = (nblk >= 2 && cv) ? s.X[(nblk - 2) * nb + c] : 0.0;
    for (int t0 = 0; t0 <= nblk - 2; t0 += RING) {
#pragma unroll
      for (int q = 0; q < RING; ++q) {
        const int j = nblk - 2 - (t0 + q);
        if (j >= 0) {
          double* zb = z + (j & 1) * NBW;
          if (h == 0) zb[c] = cv ? tj * xnext : 0.0;
          __builtin_amdgcn_wave_barrier();
          const double wcur = wj;
          tj = (j >= 1 && cv) ? s.Tn[(j - 1) * nb + c] : 0.0;
          wj = (j >= 1 && cv) ? s.X[(j - 1) * nb + c] : 0.0;
          xnext = wcur + wgemv2(w[q], zb);
          if (h == 0 && cv) s.X[j * nb + c] = xnext;
          if (j - RING >= 0) wload_block(src, (j - RING), w[q]);
        }
      }
    }
  }
  wsync();
}

// ------------------------------------------------------------------ kernels

// Steps 1-2: factor the oversampled box, solve every seed, extract
// u and phi on Gamma_i and the restriction to Omega_i.
__global__ void __launch_bounds__(64) k_basis_w(Geo g, const Box* __restrict__ boxes,
                                                const Seed* __restrict__ seeds,
                                                const double* __restrict__ K, double beta,
                                                double* __restrict__ fac,
                                                double* __restrict__ tcoup,
                                                double* __restrict__ Pk,
                                                double* __restrict__ tr_u,
                                                double* __restrict__ tr_phi,
                                                double* __restrict__ tr_beta, int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ WaveSmem sm;
  const Box B = boxes[blockIdx.x];
  const int L = lane_id();
  if (L == 0) sm.flag = 0;
  const int nrhs = B.nrhs;
  BoxLds s = carve(dsm, B, nrhs);
  load_box(g, B, K, beta, s);
  const int nc = B.ncell;
  for (int e = L; e < nrhs * nc; e += 64) s.X[e] = 0.0;
  wsync();
  for (int k = 0; k < nrhs; ++k) {
    const Seed sd = seeds[B.seed0 + k];
    const int a = sd.side >> 1, so = sd.side & 1;
    const int nf = (a == 0) ? s.m1 : s.m0;
    #pragma unroll 1
    for (int t = L; t < nf; t += 64) {
      int c[3];
      if (a == 0) { c[0] = so ? B.hi[0] - 1 : B.lo[0]; c[1] = B.lo[1] + t; }
      else { c[1] = so ? B.hi[1] - 1 : B.lo[1]; c[0] = B.lo[0] + t; }
      c[2] = 0;
      const int ox = c[0] + (a == 0 ? (so ? 1 : -1) : 0), oy = c[1] + (a == 1 ? (so ? 1 : -1) : 0);
      const double kc = kat(s, B, c[0], c[1]);
      const double bt = robin_beta(g, a, kc, kat(s, B, ox, oy), beta);
      s.X[k * nc + bloc(B, s, c[0], c[1])] = robin_T(g, kc, bt) * seed_value(g, sd, B.lo, B.hi, c);
    }
  }
  wsync();
  double* Wg = fac + B.fac;
  factor_forward(B, Wg, tcoup + B.scr, nrhs, s, sm);
  backward_cached(B, Wg, nrhs, s);
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
  wsync();
  if (L == 0 && sm.flag) atomicOr(flags, sm.flag);
}

// Step 4: particular problem on Omega_i with zero Robin data on Gamma_i.
__global__ void __launch_bounds__(64) k_particular_w(Geo g, const Box* __restrict__ boxes,
                                                     const double* __restrict__ K,
                                                     const double* __restrict__ f,
                                                     const double* __restrict__ bcv, double beta,
                                                     double* __restrict__ fac,
                                                     double* __restrict__ tcoup,
                                                     double* __restrict__ pbar,
                                                     double* __restrict__ ubar,
                                                     double* __restrict__ pibar, int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ WaveSmem sm;
  const Box B = boxes[blockIdx.x];
  const int L = lane_id();
  if (L == 0) sm.flag = 0;
  BoxLds s = carve(dsm, B, 1);
  load_box(g, B, K, beta, s);
  physical_rhs(g, B, s, f, bcv, s.X);
  wsync();
  double* Wg = fac + B.fac;
  factor_forward(B, Wg, tcoup + B.scr, 1, s, sm);
  backward_cached(B, Wg, 1, s);
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
  wsync();
  if (L == 0 && sm.flag) atomicOr(flags, sm.flag);
}

// Steps 6-7: one color phase of the smoothing sweep.  NT threads per box
// (64, 128 or 256, chosen by the autotuner) stage the box's data, build the
// right-hand side and write the outputs; the first wave runs the block
// sweeps.  The result does not depend on NT.
template <int NT>
__global__ void __launch_bounds__(NT) k_smooth_w(Geo g, const Box* __restrict__ boxes,
                                                 const int* __restrict__ members,
                                                 const double* __restrict__ K,
                                                 const double* __restrict__ f,
                                                 const double* __restrict__ bcv, double beta,
                                                 const double* __restrict__ fac,
                                                 const double* __restrict__ tcoup,
                                                 double* __restrict__ p,
                                                 double* __restrict__ gflux) {
  extern __shared__ __align__(16) double dsm[];
  const Box B = boxes[members[blockIdx.x]];
  SmoothLds r = carve_smooth(dsm, B);
  stage_smooth<NT>(g, B, r, K, p, f, gflux, bcv, tcoup);
  bsync<NT>();
  smooth_rhs<NT>(g, B, r, beta, r.b.X);
  if (threadIdx.x < 64) sweep1(B, fac + B.fac, r.b, r.b.Z);
  bsync<NT>();
  smooth_out<NT>(g, B, r, r.b.X, beta, p, gflux);
}

template <typename KF>
hipError_t set_lds(KF kern, size_t bytes) {
  if (bytes > 64 * 1024)
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
  return hipSuccess;
}

}  // namespace

size_t wave_lds_bytes(int m0, int m1, int nrhs) {
  return sizeof(double) * box_lds_doubles(m0, m1, nrhs);
}

size_t wave_smooth_lds_bytes(int m0, int m1) { return sizeof(double) * smooth_lds_doubles(m0, m1); }

hipError_t launch_basis_w(const Geo& g, const Box* boxes, int nbox, const Seed* seeds,
                          const double* K, double beta, double* fac, double* tcoup, double* scr,
                          double* Pk, double* tr_u, double* tr_phi, double* tr_beta, int* flags,
                          size_t lds, hipStream_t s) {
  (void)scr;
  if (nbox <= 0) return hipSuccess;
  hipError_t e = set_lds(k_basis_w, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_basis_w, dim3(nbox), dim3(64), lds, s, g, boxes, seeds, K, beta, fac, tcoup,
                     Pk, tr_u, tr_phi, tr_beta, flags);
  return hipGetLastError();
}

hipError_t launch_particular_w(const Geo& g, const Box* boxes, int nbox, const double* K,
                               const double* f, const double* bcv, double beta, double* fac,
                               double* tcoup, double* scr, double* pbar, double* ubar,
                               double* pibar, int* flags, size_t lds, hipStream_t s) {
  (void)scr;
  if (nbox <= 0) return hipSuccess;
  hipError_t e = set_lds(k_particular_w, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_particular_w, dim3(nbox), dim3(64), lds, s, g, boxes, K, f, bcv, beta, fac,
                     tcoup, pbar, ubar, pibar, flags);
  return hipGetLastError();
}

hipError_t launch_smooth_w(const Geo& g, const Box* boxes, const int* members, int nmem,
                           const double* K, const double* f, const double* bcv, double beta,
                           const double* fac, const double* tcoup, double* scr, double* p,
                           double* gflux, size_t lds, int nt, hipStream_t s) {
  (void)scr;
  if (nmem <= 0) return hipSuccess;
  hipError_t e;
#define MRCM_SMOOTH_NT(N)                                                                     \
  e = set_lds(k_smooth_w<N>, lds);                                                            \
  if (e != hipSuccess) return e;                                                              \
  hipLaunchKernelGGL(k_smooth_w<N>, dim3(nmem), dim3(N), lds, s, g, boxes, members, K, f, bcv, \
                     beta, fac, tcoup, p, gflux);
  if (nt == 64) {
    MRCM_SMOOTH_NT(64)
  } else if (nt == 128) {
    MRCM_SMOOTH_NT(128)
  } else if (nt == 256) {
    MRCM_SMOOTH_NT(256)
  } else {
    return hipErrorInvalidValue;
  }
#undef MRCM_SMOOTH_NT
  return hipGetLastError();
}

}  // namespace mrcm
