// Interface system (Algorithm 1, Step 5) by block cyclic reduction.
//
// With the rows of every coarse interface split between its two subdomains
// (flux rows to the lower-indexed one, pressure rows to the higher one),
// each subdomain owns as many equations as it has seed unknowns, and the
// system is block tridiagonal over the layers of subdomains along the last
// axis:  L_k x_{k-1} + D_k x_k + U_k x_{k+1} = r_k.  Odd-even reduction
// eliminates every other layer per level; all blocks of one level are
// independent, so a level is one batched dense inverse, one batch of block
// products for the eliminated layers and one for the kept layers.  No
// pivoting is used, neither across nor inside blocks (Gauss-Jordan
// inverses of the diagonal blocks).
//
// Storage: every block is dense row-major bp x bp (bp = largest layer size,
// padded layers carry the identity in D and zeros elsewhere), in one pool
// of 5M blocks (initially [D | L | U], then the reduced blocks and the
// factors F, G kept for the back substitution in slots the host schedule
// assigns) and a pool of 3M vectors [r | g | x].
#include "mrcm_internal.h"

namespace mrcm {
namespace {

// ------------------------------------------------------------------ inverse
// In-place Gauss-Jordan inversion of one bp x bp block per workgroup; each
// thread holds an 8 x 8 tile in registers; the pivot row and column go
// through LDS (double buffered: one barrier per pivot), interleaved so that
// the 16-byte pieces read by neighbouring threads are adjacent (no bank
// conflicts).  The generic update
// is a rank-1 FMA on every tile; the owners of the pivot row / column then
// overwrite those entries (uniform per unrolled pivot, so no selects).
constexpr int IT = 8;

// Reciprocal by the hardware estimate refined with two Newton steps (the
// pivots are normal numbers; the result is within an ulp of 1/x).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_bcr_inv(double* __restrict__ pool,
                                                const long long* __restrict__ offs, int bp, int ld,
                                                int* flags) {
  __shared__ __align__(16) double rowb[2][kBcrInvMax];
  __shared__ __align__(16) double colb[2][kBcrInvMax];
  __shared__ double ipb[2];
  double* A = pool + offs[blockIdx.x];
  const int nt = bp / IT;  // tiles per dimension
  const int t = threadIdx.x;
  const bool act = t < nt * nt;
  const int tr = act ? t / nt : -1, tc = act ? t - (t / nt) * nt : -1;
  const int r0 = tr * IT, c0 = tc * IT;
  double w[IT][IT];
  if (act) {
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const double2* src = reinterpret_cast<const double2*>(A + (long long)(r0 + i) * ld + c0);
#pragma unroll
      for (int j = 0; j < IT / 2; ++j) {
        const double2 v = src[j];
        w[i][2 * j] = v.x;
        w[i][2 * j + 1] = v.y;
      }
    }
  }
  int bad = 0;
  for (int kb = 0; kb < nt; ++kb) {
    const bool own_r = tr == kb, own_c = tc == kb;
#pragma unroll
    for (int kk = 0; kk < IT; ++kk) {
      double* rk = rowb[kk & 1];
      double* ck = colb[kk & 1];
      if (own_r) {
        double2* d = reinterpret_cast<double2*>(rk);
#pragma unroll
        for (int j = 0; j < IT / 2; ++j) d[j * nt + tc] = make_double2(w[kk][2 * j], w[kk][2 * j + 1]);
        if (own_c) {
          const double piv = w[kk][kk];
          bad |= !(piv != 0.0);
          ipb[kk & 1] = recip(piv);
        }
      }
      if (own_c) {
        double2* d = reinterpret_cast<double2*>(ck);
#pragma unroll
        for (int i = 0; i < IT / 2; ++i) d[i * nt + tr] = make_double2(w[2 * i][kk], w[2 * i + 1][kk]);
      }
      __syncthreads();
      if (!act) continue;
      const double ip = ipb[kk & 1];
      double rv[IT], cv[IT];
      const double2* rs = reinterpret_cast<const double2*>(rk);
      const double2* cs = reinterpret_cast<const double2*>(ck);
#pragma unroll
      for (int j = 0; j < IT / 2; ++j) {
        const double2 a = rs[j * nt + tc], b = cs[j * nt + tr];
        rv[2 * j] = a.x;
        rv[2 * j + 1] = a.y;
        cv[2 * j] = -b.x * ip;
        cv[2 * j + 1] = -b.y * ip;
      }
#pragma unroll
      for (int i = 0; i < IT; ++i)
#pragma unroll
        for (int j = 0; j < IT; ++j) w[i][j] = fma(cv[i], rv[j], w[i][j]);
      if (own_r) {
#pragma unroll
        for (int j = 0; j < IT; ++j) w[kk][j] = rv[j] * ip;
      }
      if (own_c) {
#pragma unroll
        for (int i = 0; i < IT; ++i) w[i][kk] = cv[i];
        if (own_r) w[kk][kk] = ip;
      }
    }
  }
  if (act) {
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      double2* dst = reinterpret_cast<double2*>(A + (long long)(r0 + i) * ld + c0);
#pragma unroll
      for (int j = 0; j < IT / 2; ++j) dst[j] = make_double2(w[i][2 * j], w[i][2 * j + 1]);
    }
  }
  if (bad) atomicOr(flags, kFlagSingular);
}

// ------------------------------------------------------------------ products
// C = [C0] + al1 A1 B1 + al2 A2 B2 for a batch of tasks; the operands are
// n x n matrices at element offsets in the pool with leading dimension ld
// (whole blocks, or quarters of a block in the two-by-two inverse).  One
// workgroup of 256 threads per 32 x 32 output tile; the whole 32 x n strip
// of A (transposed, k-major) and n x 32 strip of B are staged in LDS with
// all global loads of a chunk in flight before the stores; each thread
// computes a 2 x 2 set of outputs.
constexpr int GT = 32, GCH = 16;

__device__ __forceinline__ void stage_strips(const double* __restrict__ A, const double* __restrict__ B,
                                             double al, int n, int ld, int tr0, int tc0, double* As,
                                             double* Bs) {
  // As[k * GT + r] = al * A[tr0 + r][k];  Bs[k * GT + c] = B[k][tc0 + c]
  const int cnt = GT * n;  // elements per strip
  for (int e0 = 0; e0 < cnt; e0 += 256 * GCH) {
    double va[GCH], vb[GCH];
#pragma unroll
    for (int u = 0; u < GCH; ++u) {
      const int e = e0 + u * 256 + threadIdx.x;
      const bool ok = e < cnt;
      const int ra = e / n, ka = e - (e / n) * n;  // A row-major: consecutive k
      const int kb = e >> 5, cb = e & 31;          // B: 32 consecutive columns
      va[u] = ok ? A[(long long)(tr0 + ra) * ld + ka] : 0.0;
      vb[u] = ok ? B[(long long)kb * ld + tc0 + cb] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < GCH; ++u) {
      const int e = e0 + u * 256 + threadIdx.x;
      if (e < cnt) {
        const int ra = e / n, ka = e - (e / n) * n;
        As[ka * GT + ra] = al * va[u];
        Bs[e] = vb[u];
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_bcr_gemm(double* __restrict__ pool,
                                                  const BcrGemm* __restrict__ tasks, int n, int ld) {
  extern __shared__ double smem[];
  double* As = smem;           // n x GT
  double* Bs = smem + n * GT;  // n x GT
  const int ntile = n / GT;
  const int task = blockIdx.x / (ntile * ntile);
  const int tile = blockIdx.x - task * ntile * ntile;
  const BcrGemm T = tasks[task];
  const int tr0 = (tile / ntile) * GT, tc0 = (tile % ntile) * GT;
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  double acc00 = 0.0, acc01 = 0.0, acc10 = 0.0, acc11 = 0.0;
  for (int term = 0; term < 2; ++term) {
    const long long ai = term ? T.a2 : T.a1, bi = term ? T.b2 : T.b1;
    if (ai < 0) continue;
    if (term) __syncthreads();
    stage_strips(pool + ai, pool + bi, term ? T.al2 : T.al1, n, ld, tr0, tc0, As, Bs);
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < n; ++k) {
      const double a0 = As[k * GT + ty], a1 = As[k * GT + ty + 16];
      const double b0 = Bs[k * GT + tx], b1 = Bs[k * GT + tx + 16];
      acc00 = fma(a0, b0, acc00);
      acc01 = fma(a0, b1, acc01);
      acc10 = fma(a1, b0, acc10);
      acc11 = fma(a1, b1, acc11);
    }
  }
  double* C = pool + T.c;
  const double* C0 = T.c0 >= 0 ? pool + T.c0 : nullptr;
  const long long r_0 = tr0 + ty, r_1 = r_0 + 16;
  const int c_0 = tc0 + tx, c_1 = c_0 + 16;
  if (C0) {
    acc00 += C0[r_0 * ld + c_0];
    acc01 += C0[r_0 * ld + c_1];
    acc10 += C0[r_1 * ld + c_0];
    acc11 += C0[r_1 * ld + c_1];
  }
  C[r_0 * ld + c_0] = acc00;
  C[r_0 * ld + c_1] = acc01;
  C[r_1 * ld + c_0] = acc10;
  C[r_1 * ld + c_1] = acc11;
}

// y = [y0] + al1 A1 x1 + al2 A2 x2.  Workgroup (task, group of 16 rows);
// 16 lanes per row, each with bp/16 independent loads, then a 16-lane sum.
__global__ void __launch_bounds__(256) k_bcr_gemv(const double* __restrict__ pool,
                                                  double* __restrict__ vec,
                                                  const BcrGemv* __restrict__ tasks, int bp) {
  const BcrGemv T = tasks[blockIdx.x];
  const long long bs = (long long)bp * bp;
  const int r = blockIdx.y * 16 + (threadIdx.x >> 4), l = threadIdx.x & 15;
  double acc = 0.0;
#pragma unroll
  for (int term = 0; term < 2; ++term) {
    const int ai = term ? T.a2 : T.a1;
    if (ai < 0) continue;
    const double* A = pool + ai * bs + (long long)r * bp;
    const double* x = vec + (long long)(term ? T.x2 : T.x1) * bp;
    double s = 0.0;
#pragma unroll 4
    for (int c = l; c < bp; c += 16) s = fma(A[c], x[c], s);
    acc = fma(term ? T.al2 : T.al1, s, acc);
  }
  acc += __shfl_xor(acc, 8);
  acc += __shfl_xor(acc, 4);
  acc += __shfl_xor(acc, 2);
  acc += __shfl_xor(acc, 1);
  if (l == 0) {
    double* y = vec + (long long)T.y * bp;
    y[r] = (T.y0 >= 0 ? vec[(long long)T.y0 * bp + r] : 0.0) + acc;
  }
}

// Scatter the interface system assembled in band form into the dense
// layer blocks: row-band RB (row i, column c at RB[i*(kl+ku+1) + c-i+kl]),
// right-hand side rhs; row_lvl/row_loc and col_lvl/col_loc map an equation
// and an unknown to its layer and position; padding gets the identity.
__global__ void k_bcr_scatter(const double* __restrict__ RB, const double* __restrict__ rhs, int n,
                              int kl, int ku, const int* __restrict__ row_lvl,
                              const int* __restrict__ row_loc, const int* __restrict__ col_lvl,
                              const int* __restrict__ col_loc, int M, int bp,
                              double* __restrict__ pool, double* __restrict__ vec) {
  const int W = kl + ku + 1;
  const long long bs = (long long)bp * bp;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * W) return;
  const int i = (int)(e / W), t = (int)(e - (long long)i * W);
  const int c = i - kl + t;
  const int li = row_lvl[i], ri = row_loc[i];
  if (t == 0) vec[(long long)li * bp + ri] = rhs[i];
  if (c < 0 || c >= n) return;
  const double v = RB[e];
  if (v == 0.0) return;
  const int lc = col_lvl[c], rc = col_loc[c];
  int kind;
  if (lc == li) kind = 0;
  else if (lc == li - 1) kind = 1;
  else kind = 2;  // lc == li + 1 (block tridiagonal by construction)
  pool[(long long)(kind * M + li) * bs + (long long)ri * bp + rc] = v;
}

// Identity on the padded diagonal of every D block.
__global__ void k_bcr_pad(double* __restrict__ pool, const int* __restrict__ lsize, int bp) {
  const int k = blockIdx.x;
  const long long bs = (long long)bp * bp;
  for (int r = lsize[k] + threadIdx.x; r < bp; r += blockDim.x) pool[k * bs + (long long)r * bp + r] = 1.0;
}

// x (layer-major, padded) -> X (unknown order).
__global__ void k_bcr_gather(const double* __restrict__ xv, const int* __restrict__ col_lvl,
                             const int* __restrict__ col_loc, int n, int bp, double* __restrict__ X) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) X[c] = xv[(long long)col_lvl[c] * bp + col_loc[c]];
}

}  // namespace

hipError_t launch_bcr_inv(double* pool, const long long* offs, int nblk, int n, int ld, int* flags,
                          hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  if (n % IT || n > kBcrInvMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bcr_inv<256>, dim3(nblk), dim3(256), 0, s, pool, offs, n, ld, flags);
  return hipGetLastError();
}

hipError_t launch_bcr_gemm(double* pool, const BcrGemm* tasks, int ntask, int n, int ld, hipStream_t s) {
  if (ntask <= 0) return hipSuccess;
  if (n % GT || n > kBcrMaxBlock) return hipErrorInvalidValue;
  const int ntile = n / GT;
  const size_t lds = 2 * sizeof(double) * (size_t)n * GT;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_bcr_gemm,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_bcr_gemm, dim3(ntask * ntile * ntile), dim3(256), lds, s, pool, tasks, n, ld);
  return hipGetLastError();
}

hipError_t launch_bcr_gemv(const double* pool, double* vec, const BcrGemv* tasks, int ntask, int bp,
                           hipStream_t s) {
  if (ntask <= 0) return hipSuccess;
  if (bp % 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bcr_gemv, dim3(ntask, bp / 16), dim3(256), 0, s, pool, vec, tasks, bp);
  return hipGetLastError();
}

hipError_t launch_bcr_scatter(const double* RB, const double* rhs, int n, int kl, int ku,
                              const int* row_lvl, const int* row_loc, const int* col_lvl,
                              const int* col_loc, int M, int bp, double* pool, double* vec,
                              const int* lsize, hipStream_t s) {
  const long long tot = (long long)n * (kl + ku + 1);
  hipLaunchKernelGGL(k_bcr_scatter, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, RB, rhs, n,
                     kl, ku, row_lvl, row_loc, col_lvl, col_loc, M, bp, pool, vec);
  hipLaunchKernelGGL(k_bcr_pad, dim3(M), dim3(64), 0, s, pool, lsize, bp);
  return hipGetLastError();
}

hipError_t launch_bcr_pad(double* pool, const int* lsize, int M, int bp, hipStream_t s) {
  hipLaunchKernelGGL(k_bcr_pad, dim3(M), dim3(64), 0, s, pool, lsize, bp);
  return hipGetLastError();
}

hipError_t launch_bcr_gather(const double* xv, const int* col_lvl, const int* col_loc, int n, int bp,
                             double* X, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bcr_gather, dim3((n + 255) / 256), dim3(256), 0, s, xv, col_lvl, col_loc, n, bp, X);
  return hipGetLastError();
}

}  // namespace mrcm
