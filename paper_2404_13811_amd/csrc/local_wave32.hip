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
#include "wave32_common.h"

namespace mrcm {
namespace {

using namespace wave;

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
  BoxR R = carve_r(dsm, B, max(nrhs, 1), 0, g.kc);
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
      const double kc = kat(s, B, x, y, a), ko = kat(s, B, ox, oy, a);
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
  BoxR R = carve_r(dsm, B, 1, 1, g.kc);
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
      const double kc = kat(s, B, x, y, a);
      const double bt = robin_beta(g, a, kc, kat(s, B, ox, oy, a), beta);
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
  SmoothLds r = carve_smooth(dsm, B, g.kc);
  BoxR R = carve_smooth_r(dsm, r);
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

size_t wave32_lds_bytes(int m0, int m1, int nrhs, int nbrhs, int kc) {
  return boxr_bytes(m0, m1, nrhs, nbrhs, kc);
}

size_t wave32_smooth_lds_bytes(int m0, int m1, int kc) { return smooth32_lds_bytes(m0, m1, kc); }

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
