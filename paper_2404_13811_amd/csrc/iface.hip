// Interface system of MRCM-O on gfx950 (Algorithm 1, Steps 3-5).
//
// Unknowns X_i^k (subdomain-major, seeds in side order).  For every coarse
// interface Gamma_ij (i < j) and every test function mu of M_H (resp. V_H)
// on it, one flux row and one pressure row (equations int_ujump, int_pjump):
//   sum_e |e| mu (sum_k X_i^k u_i^k + sum_k X_j^k u_j^k) = -sum_e |e| mu (ubar_i + ubar_j)
//   sum_e |e| mu (sum_k X_i^k (beta u_i^k + phi_i^k) - sum_k X_j^k (...))
//                                                        = -sum_e |e| mu (beta ubar_i - beta ubar_j)
// (the unique normal points out of the lower index, hence +/-).  The system
// is banded in this ordering; it is assembled straight into LAPACK-style
// band storage and solved by one workgroup with partial pivoting whose
// active (kl+1) x (kl+ku+1) window lives in LDS.
#include "local_common.h"

namespace mrcm {
namespace {

__device__ __forceinline__ void omega_box(const Geo& g, int sub, int lo[3], int hi[3]) {
  int r = sub;
  for (int a = 0; a < 3; ++a) {
    const int Ma = (a < g.d) ? g.M[a] : 1;
    const int ia = r % Ma;
    r /= Ma;
    lo[a] = (a < g.d) ? ia * g.S[a] : 0;
    hi[a] = (a < g.d) ? lo[a] + g.S[a] : 1;
  }
}

__device__ __forceinline__ void gface_cell(const int lo[3], const int hi[3], int q, int t, int c[3]) {
  const int a = q >> 1, s = q & 1;
  int r = t;
  for (int b = 0; b < 3; ++b) {
    if (b == a) {
      c[b] = s ? hi[b] - 1 : lo[b];
    } else {
      const int m = hi[b] - lo[b];
      c[b] = lo[b] + r % m;
      r /= m;
    }
  }
}

// One workgroup per interface; threads over (row, entry) pairs.
__global__ void k_moments(Geo g, const Iface* __restrict__ ifc, const Seed* __restrict__ basis,
                          const int* __restrict__ seed_off, const double* __restrict__ tr_u,
                          const double* __restrict__ tr_phi, const double* __restrict__ tr_beta,
                          const double* __restrict__ ubar, const double* __restrict__ pibar,
                          double* __restrict__ AB, int ldab, int kl, int ku,
                          double* __restrict__ rhs) {
  const Iface F = ifc[blockIdx.x];
  const int qi = 2 * F.axis + 1, qj = 2 * F.axis;
  const int ni = seed_off[F.i + 1] - seed_off[F.i];
  const int nj = seed_off[F.j + 1] - seed_off[F.j];
  const int per_row = ni + nj + 1;  // entries + rhs
  const int nrow = 2 * F.nbasis;
  int ilo[3], ihi[3];
  omega_box(g, F.i, ilo, ihi);
  int nf = 1;
  for (int b = 0; b < g.d; ++b)
    if (b != F.axis) nf *= g.S[b];
  for (int w = threadIdx.x; w < nrow * per_row; w += blockDim.x) {
    const int rr = w / per_row, e = w % per_row;
    const int kind = rr / F.nbasis;  // 0 flux, 1 pressure
    const Seed mu = basis[F.basis0 + rr % F.nbasis];
    const int row = F.row0 + rr;
    double acc = 0.0;
    int col = -1;
    if (e < ni + nj) {
      const bool side_i = e < ni;
      const int sub = side_i ? F.i : F.j;
      const int k = side_i ? e : e - ni;
      const int q = side_i ? qi : qj;
      const double sg = (kind == 1 && !side_i) ? -1.0 : 1.0;
      col = seed_off[sub] + k;
      const long long base = (long long)col * g.gstride + g.gside_off[q];
      const long long bbase = (long long)sub * g.gstride + g.gside_off[q];
      for (int t = 0; t < nf; ++t) {
        int c[3];
        gface_cell(ilo, ihi, qi, t, c);
        const double w_t = g.area * seed_value(g, mu, ilo, ihi, c);
        const double v = kind == 0 ? tr_u[base + t] : tr_beta[bbase + t] * tr_u[base + t] + tr_phi[base + t];
        acc += w_t * v;
      }
      acc *= sg;
      if (g.neumann && row == 0) acc = (col == 0) ? 1.0 : 0.0;
      AB[(long long)col * ldab + (kl + ku + row - col)] = acc;
    } else {
      const long long bi = (long long)F.i * g.gstride + g.gside_off[qi];
      const long long bj = (long long)F.j * g.gstride + g.gside_off[qj];
      for (int t = 0; t < nf; ++t) {
        int c[3];
        gface_cell(ilo, ihi, qi, t, c);
        const double w_t = g.area * seed_value(g, mu, ilo, ihi, c);
        const double v = kind == 0 ? ubar[bi + t] + ubar[bj + t] : pibar[bi + t] - pibar[bj + t];
        acc += w_t * v;
      }
      rhs[row] = (g.neumann && row == 0) ? 0.0 : -acc;
    }
  }
}

constexpr int LU_THREADS = 1024;

// Banded LU with partial pivoting on rows j..j+kl, forward elimination of
// the right-hand side carried along, U rows written back over AB, then
// back substitution.  One workgroup; LDS holds the active window.
__global__ void __launch_bounds__(LU_THREADS) k_bandlu(double* __restrict__ AB, int ldab, int n,
                                                       int kl, int ku,
                                                       const double* __restrict__ rhs,
                                                       double* __restrict__ x, int* flags) {
  extern __shared__ double smem[];
  const int R = kl + 1;
  const int CW = kl + ku + 1;
  double* win = smem;              // R * CW
  double* zr = win + R * CW;       // R
  double* lm = zr + R;             // R (multipliers)
  __shared__ int s_piv;
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  if (tid == 0) s_flag = 0;
  auto W = [&](int i, int c) -> double& { return win[(i % R) * CW + (c % CW)]; };
  auto orig = [&](int i, int c) -> double {
    if (c < 0 || c >= n || i < 0 || i >= n) return 0.0;
    if (c - i > ku || i - c > kl) return 0.0;
    return AB[(long long)c * ldab + (kl + ku + i - c)];
  };
  // initial window: rows 0..kl, cols 0..kl+ku
  for (int e = tid; e < R * CW; e += LU_THREADS) {
    const int i = e / CW, c = e % CW;
    W(i, c) = orig(i, c);
  }
  for (int i = tid; i < R; i += LU_THREADS) zr[i % R] = (i < n) ? rhs[i] : 0.0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int km = min(kl, n - 1 - j);
    // pivot search (wave 0)
    if (tid < 64) {
      double best = -1.0;
      int bi = j;
      for (int t = tid; t <= km; t += 64) {
        const double v = fabs(W(j + t, j));
        if (v > best) { best = v; bi = j + t; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) {
        s_piv = bi;
        if (!(best > 0.0)) s_flag |= kFlagSingular;
      }
    }
    __syncthreads();
    const int pr = s_piv;
    if (pr != j) {
      for (int c = tid; c < CW; c += LU_THREADS) {
        const double a = W(j, j + c);
        W(j, j + c) = W(pr, j + c);
        W(pr, j + c) = a;
      }
      if (tid == 0) {
        const double a = zr[j % R];
        zr[j % R] = zr[pr % R];
        zr[pr % R] = a;
      }
    }
    __syncthreads();
    const double piv = W(j, j);
    for (int i = 1 + tid; i <= km; i += LU_THREADS) lm[i] = (piv != 0.0) ? W(j + i, j) / piv : 0.0;
    __syncthreads();
    // rank-1 update of rows j+1..j+km, columns j+1..j+kl+ku; rhs too
    const int ncols = CW - 1;
    for (int e = tid; e < km * (ncols + 1); e += LU_THREADS) {
      const int i = 1 + e / (ncols + 1), c = e % (ncols + 1);
      if (c < ncols) W(j + i, j + 1 + c) -= lm[i] * W(j, j + 1 + c);
      else zr[(j + i) % R] -= lm[i] * zr[j % R];
    }
    // U row j back to AB (band position of A(j, j + c))
    for (int c = tid; c < CW; c += LU_THREADS) {
      if (j + c < n) AB[(long long)(j + c) * ldab + (kl + ku - c)] = W(j, j + c);
    }
    __syncthreads();
    if (tid == 0) x[j] = zr[j % R];  // forward-eliminated rhs, solved in place below
    // slide the window: row j -> row j + kl + 1, column j -> column j + CW
    const int nr = j + kl + 1;
    for (int c = tid; c < CW; c += LU_THREADS) W(nr, j + 1 + c) = (nr < n) ? orig(nr, j + 1 + c) : 0.0;
    if (tid == 0) zr[nr % R] = (nr < n) ? rhs[nr] : 0.0;
    for (int i = 1 + tid; i <= kl; i += LU_THREADS) W(j + i, j + CW) = 0.0;
    __syncthreads();
  }
  // back substitution with U (upper bandwidth kl + ku), wave 0
  double* xs = smem;  // circular buffer of the last CW solutions
  __syncthreads();
  if (tid < 64) {
    for (int j = n - 1; j >= 0; --j) {
      double acc = 0.0;
      for (int c = 1 + tid; c < CW; c += 64)
        if (j + c < n) acc += AB[(long long)(j + c) * ldab + (kl + ku - c)] * xs[(j + c) % CW];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      const double u = AB[(long long)j * ldab + (kl + ku)];
      const double v = (x[j] - acc) / u;
      if (tid == 0) {
        xs[j % CW] = v;
        x[j] = v;
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  if (tid == 0 && s_flag) atomicOr(flags, s_flag);
}

// MRCM-O assembly: p = pbar + sum_k X_k P_k on each Omega_i and Gamma fluxes
// u = ubar + sum_k X_k u_k (equations eq:addu, eq:addp, eq:uhatphat).
__global__ void k_combine_p(Geo g, const int* __restrict__ seed_off, const double* __restrict__ X,
                            const double* __restrict__ Pk, const double* __restrict__ pbar,
                            double* __restrict__ p) {
  const int ncell_o = g.S[0] * g.S[1] * (g.d == 3 ? g.S[2] : 1);
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)g.nsub * ncell_o) return;
  const int sub = (int)(e / ncell_o), t = (int)(e % ncell_o);
  double v = pbar[e];
  for (int k = seed_off[sub]; k < seed_off[sub + 1]; ++k) v += X[k] * Pk[(long long)k * ncell_o + t];
  int lo[3], hi[3];
  omega_box(g, sub, lo, hi);
  const int c0 = lo[0] + t % g.S[0];
  const int c1 = lo[1] + (t / g.S[0]) % g.S[1];
  const int c2 = (g.d == 3) ? lo[2] + t / (g.S[0] * g.S[1]) : 0;
  p[c0 + g.n[0] * (c1 + g.n[1] * c2)] = v;
}

__global__ void k_combine_u(Geo g, const int* __restrict__ seed_off, const double* __restrict__ X,
                            const double* __restrict__ tr_u, const double* __restrict__ ubar,
                            double* __restrict__ gflux) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)g.nsub * g.gstride) return;
  const int sub = (int)(e / g.gstride), t = (int)(e % g.gstride);
  double v = ubar[e];
  for (int k = seed_off[sub]; k < seed_off[sub + 1]; ++k) v += X[k] * tr_u[(long long)k * g.gstride + t];
  gflux[e] = v;
}

}  // namespace

hipError_t launch_moments(const Geo& g, const Iface* ifc, int nifc, const Seed* basis,
                          const int* seed_off, const double* tr_u, const double* tr_phi,
                          const double* tr_beta, const double* ubar, const double* pibar,
                          double* AB, int ldab, int kl, int ku, double* rhs, hipStream_t s) {
  if (nifc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_moments, dim3(nifc), dim3(64), 0, s, g, ifc, basis, seed_off, tr_u, tr_phi,
                     tr_beta, ubar, pibar, AB, ldab, kl, ku, rhs);
  return hipGetLastError();
}

hipError_t launch_bandlu_solve(double* AB, int ldab, int n, int kl, int ku, double* rhs, double* x,
                               int* ipiv, int* flags, hipStream_t s) {
  (void)ipiv;
  if (n <= 0) return hipSuccess;
  const size_t lds = sizeof(double) * ((size_t)(kl + 1) * (kl + ku + 1) + 2 * (kl + 1));
  if (lds > 160 * 1024 - 64) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_bandlu,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_bandlu, dim3(1), dim3(LU_THREADS), lds, s, AB, ldab, n, kl, ku, rhs, x,
                     flags);
  return hipGetLastError();
}

hipError_t launch_combine(const Geo& g, const int* seed_off, const double* X, const double* Pk,
                          const double* tr_u, const double* pbar, const double* ubar, double* p,
                          double* gflux, hipStream_t s) {
  const int ncell_o = g.S[0] * g.S[1] * (g.d == 3 ? g.S[2] : 1);
  const long long n1 = (long long)g.nsub * ncell_o;
  hipLaunchKernelGGL(k_combine_p, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, g, seed_off,
                     X, Pk, pbar, p);
  const long long n2 = (long long)g.nsub * g.gstride;
  hipLaunchKernelGGL(k_combine_u, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, g, seed_off,
                     X, tr_u, ubar, gflux);
  return hipGetLastError();
}

}  // namespace mrcm
