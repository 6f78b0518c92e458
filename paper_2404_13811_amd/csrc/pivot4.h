// A 4 x 4 pivot block of block Gauss-Jordan elimination without pivoting:
// P = [[a, b], [e, d]] in 2 x 2 blocks, factored by the block elimination
//   y = a^{-1} r1,  E = a^{-1} b,  S = d - e E,  v2 = S^{-1} (r2 - e y),
//   v1 = y - E v2,
// so that v = P^{-1} r.  The 2 x 2 inverses use their closed form (one
// reciprocal each), which keeps the dependent chain short.  The four
// pivots of the equivalent scalar elimination are P00, det(a) / P00, S00
// and det(S) / S00; callers test them through d0, da, s0, ds.
#pragma once
#include <hip/hip_runtime.h>

namespace mrcm {

__device__ __forceinline__ double pivot_rcp(double x) {
  // hardware estimate refined by two Newton steps (within an ulp of 1/x)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float pivot_rcp(float x) { return 1.0f / x; }

// a pivot the elimination can divide by: finite and non-zero
template <typename T>
__device__ __forceinline__ bool piv_usable(T x) {
  return x == x && x != T(0) && x - x == T(0);
}

template <typename T>
struct PivBlock {
  T ai[2][2], E[2][2], e[2][2], si[2][2];
  T d0, da, s0, ds;  // P00, det(a), S00, det(S)
};

template <typename T>
__device__ __forceinline__ PivBlock<T> piv_block(const T P[4][4]) {
  PivBlock<T> q;
  const T da = P[0][0] * P[1][1] - P[0][1] * P[1][0];
  const T ia = pivot_rcp(da);
  q.ai[0][0] = P[1][1] * ia;
  q.ai[0][1] = -P[0][1] * ia;
  q.ai[1][0] = -P[1][0] * ia;
  q.ai[1][1] = P[0][0] * ia;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      q.E[i][j] = q.ai[i][0] * P[0][2 + j] + q.ai[i][1] * P[1][2 + j];
      q.e[i][j] = P[2 + i][j];
    }
  T S[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) S[i][j] = P[2 + i][2 + j] - (q.e[i][0] * q.E[0][j] + q.e[i][1] * q.E[1][j]);
  const T ds = S[0][0] * S[1][1] - S[0][1] * S[1][0];
  const T is = pivot_rcp(ds);
  q.si[0][0] = S[1][1] * is;
  q.si[0][1] = -S[0][1] * is;
  q.si[1][0] = -S[1][0] * is;
  q.si[1][1] = S[0][0] * is;
  q.d0 = P[0][0];
  q.da = da;
  q.s0 = S[0][0];
  q.ds = ds;
  return q;
}

// v = P^{-1} r with the factors of piv_block
template <typename T>
__device__ __forceinline__ void piv_apply(const PivBlock<T>& q, const T r[4], T v[4]) {
  const T y0 = q.ai[0][0] * r[0] + q.ai[0][1] * r[1];
  const T y1 = q.ai[1][0] * r[0] + q.ai[1][1] * r[1];
  const T z0 = r[2] - (q.e[0][0] * y0 + q.e[0][1] * y1);
  const T z1 = r[3] - (q.e[1][0] * y0 + q.e[1][1] * y1);
  v[2] = q.si[0][0] * z0 + q.si[0][1] * z1;
  v[3] = q.si[1][0] * z0 + q.si[1][1] * z1;
  v[0] = y0 - (q.E[0][0] * v[2] + q.E[0][1] * v[3]);
  v[1] = y1 - (q.E[1][0] * v[2] + q.E[1][1] * v[3]);
}

}  // namespace mrcm
