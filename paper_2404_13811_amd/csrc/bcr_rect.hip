// Kernels of the two-level interface solver (3-D grids of subdomains whose
// layers are too large for one dense block): batched products of
// rectangular blocks on FP64 MFMA, the assembly of the reduced system over
// the gaps between outer layers from the inner solutions, and the final
// back substitution into the interface unknowns.  The block elimination
// itself (inverses, square products, block-vector products) reuses the
// cyclic-reduction kernels of bcr.hip.
#include "mrcm_internal.h"

#include <algorithm>

namespace mrcm {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int TM, int TN, int KC>
constexpr size_t rect_lds_doubles() {
  return (size_t)TM * (KC + 1) + (size_t)KC * TN;
}

// One TM x TN tile of C = [C0] + al1 A1 B1 [+ al2 A2 B2] (A: m x k with
// leading dimension lda, B: k x n with ldb, C and C0: m x n with ldc; all
// offsets into one base array).  Four waves in a 2 x 2 arrangement, each a
// (TM/2) x (TN/2) quadrant of 16 x 16 blocks on FP64 16 x 16 x 4 matrix
// instructions (lane l: A[l % 16][l / 16], B[l / 16][l % 16], result element
// r at row 4r + l / 16, column l % 16); k in chunks of KC staged in LDS with
// the next chunk's loads in flight.  A wave of a 64 x 64 tile reuses each
// operand it reads from LDS for two instructions.
template <int TM, int TN, int KC>
__device__ __forceinline__ void rect_tile_at(double* base, const BcrGemm& T, const RectShape& S,
                                             int tr0, int tc0, double* smem) {
  constexpr int NA = TM * KC / 256, NB = KC * TN / 256;
  constexpr int AS = KC + 1;
  constexpr int BM = TM / 32, BN = TN / 32;  // 16 x 16 blocks per wave
  // one block per wave: two accumulators on alternate k steps
  constexpr int NACC = BM * BN == 1 ? 2 : 1;
  double* As = smem;
  double* Bs = smem + TM * AS;
  const int tid = threadIdx.x;
  const int wv = tid >> 6, ln = tid & 63;
  const int qr = (wv >> 1) * (TM / 2), qc = (wv & 1) * (TN / 2);
  const int li = ln & 15, lk = ln >> 4;
  const int t0 = T.a1 >= 0 ? 0 : 1;
  const int nterm = (T.a1 >= 0 ? 1 : 0) + (T.a2 >= 0 ? 1 : 0);
  const int nch = S.k / KC, total = nterm * nch;
  double va[NA], vb[NB];
  auto load = [&](int c) {
    const int term = c < nch ? t0 : 1;
    const int k0 = (c % nch) * KC;
    const double* A = base + (term ? T.a2 : T.a1);
    const double* B = base + (term ? T.b2 : T.b1);
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = u * 256 + tid;
      va[u] = A[(long long)(tr0 + e / KC) * S.lda + k0 + e % KC];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = u * 256 + tid;
      vb[u] = B[(long long)(k0 + e / TN) * S.ldb + tc0 + e % TN];
    }
  };
  dbl4 acc[NACC][BM][BN];
#pragma unroll
  for (int h = 0; h < NACC; ++h)
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) acc[h][i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  if (total > 0) load(0);
  for (int c = 0; c < total; ++c) {
    const double al = (c < nch ? t0 : 1) ? T.al2 : T.al1;
    if (c) __syncthreads();
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = u * 256 + tid;
      As[(e / KC) * AS + e % KC] = al * va[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) Bs[u * 256 + tid] = vb[u];
    __syncthreads();
    if (c + 1 < total) load(c + 1);
#pragma unroll
    for (int k = 0; k < KC; k += 4) {
      double a[BM], b[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) a[i] = As[(qr + 16 * i + li) * AS + k + lk];
#pragma unroll
      for (int j = 0; j < BN; ++j) b[j] = Bs[(k + lk) * TN + qc + 16 * j + li];
      const int h = NACC == 2 ? (k / 4) & 1 : 0;
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
          acc[h][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[h][i][j], 0, 0, 0);
    }
  }
  double* C = base + T.c;
  const double* C0 = T.c0 >= 0 ? base + T.c0 : nullptr;
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int col = tc0 + qc + 16 * j + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long row = tr0 + qr + 16 * i + 4 * r + lk;
        double v = acc[0][i][j][r];
        if (NACC == 2) v += acc[NACC - 1][i][j][r];
        if (C0) v += C0[row * S.ldc + col];
        C[row * S.ldc + col] = v;
      }
    }
}

template <int TM, int TN, int KC>
__device__ __forceinline__ void rect_tile(double* base, const BcrGemm& T, const RectShape& S,
                                          int tile, double* smem) {
  const int ntc = S.n / TN;
  rect_tile_at<TM, TN, KC>(base, T, S, (tile / ntc) * TM, (tile % ntc) * TN, smem);
}

// Products restricted to their column windows: workgroup (task, row tile,
// j) takes the task's j-th window tile, or returns when the window has
// fewer than j + 1 tiles (the whole workgroup, before any barrier).
template <int TM, int TN, int KC>
__global__ void __launch_bounds__(256) k_rect_gemm_win(double* __restrict__ base,
                                                       const BcrGemm* __restrict__ tasks, RectShape S,
                                                       int maxnt) {
  extern __shared__ double smem[];
  const int per = (S.m / TM) * maxnt;
  const int task = blockIdx.x / per;
  const int loc = blockIdx.x - task * per;
  const int i = loc / maxnt, j = loc - i * maxnt;
  const BcrGemm T = tasks[task];
  int t0 = 0, t1 = S.n / TN, tx = -1;
  if (T.wc1 > 0) {
    t0 = T.wc0 / TN;
    t1 = min((T.wc1 + TN - 1) / TN, S.n / TN);
    tx = T.wcx >= 0 ? T.wcx / TN : -1;
    if (tx >= t0 && tx < t1) tx = -1;
  }
  const int cnt = (t1 - t0) + (tx >= 0 ? 1 : 0);
  if (j >= cnt) return;
  const int ct = j < t1 - t0 ? t0 + j : tx;
  rect_tile_at<TM, TN, KC>(base, T, S, i * TM, ct * TN, smem);
}

template <int TM, int TN, int KC>
__global__ void __launch_bounds__(256) k_rect_gemm(double* __restrict__ base,
                                                   const BcrGemm* __restrict__ tasks,
                                                   RectShape S) {
  extern __shared__ double smem[];
  const int per = (S.m / TM) * (S.n / TN);
  const int task = blockIdx.x / per;
  rect_tile<TM, TN, KC>(base, tasks[task], S, blockIdx.x - task * per, smem);
}

// Two independent groups of products of different shapes (and the same k)
// in one launch: the first na * (tiles of SA) workgroups take group A.
template <int TM, int TN, int KC>
__global__ void __launch_bounds__(256) k_rect_gemm2(double* __restrict__ base,
                                                    const BcrGemm* __restrict__ ta, int na, RectShape SA,
                                                    const BcrGemm* __restrict__ tb, RectShape SB) {
  extern __shared__ double smem[];
  const int pa = (SA.m / TM) * (SA.n / TN);
  int b = blockIdx.x;
  if (b < na * pa) {
    const int task = b / pa;
    rect_tile<TM, TN, KC>(base, ta[task], SA, b - task * pa, smem);
  } else {
    b -= na * pa;
    const int pb = (SB.m / TM) * (SB.n / TN);
    const int task = b / pb;
    rect_tile<TM, TN, KC>(base, tb[task], SB, b - task * pb, smem);
  }
}

// base[0, n) = 0; then (second kernel) base[ones[i]] = 1 for the listed
// offsets (identity blocks and padding, unit right-hand-side columns).
// zero nrep runs of len doubles, stride apart, from base
__global__ void k_fill_zero(double* __restrict__ base, long long len, long long stride, long long nrep) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len * nrep) return;
  const long long r = e / len;
  base[r * stride + (e - r * len)] = 0.0;
}
__global__ void k_set_ones(double* __restrict__ base, const long long* __restrict__ ones, long long nones) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nones) base[ones[e]] = 1.0;
}

// Rows of the reduced system: row q of reduced row set `set` is the sum
// over its cross entries (value at base[cval], row position ypos in the
// stacked inner solution of its source layer) of value * that solution
// row; column c of the result goes to base[dst[set] + map(c)], where the
// column map sends column 0 to the right-hand side and the coupling
// columns to their reduced blocks.  One workgroup per (row, column chunk).
__global__ void __launch_bounds__(256) k_lsc_outer_rows(double* __restrict__ base,
                                                        const LscRow* __restrict__ rows,
                                                        const long long* __restrict__ ypos,
                                                        const int* __restrict__ cmap, int nrow,
                                                        int ncol, int width) {
  const int q = blockIdx.x;
  if (q >= nrow) return;
  const LscRow R = rows[q];
  for (int c = blockIdx.y * blockDim.x + threadIdx.x; c < ncol; c += gridDim.y * blockDim.x) {
    const int code = cmap[R.cm + c];
    long long d;
    if (code == -2) d = R.rhs;
    else if (code < 0) d = -1;
    else if (code < R.ml) d = R.dst0 >= 0 ? R.dst0 + code : -1;
    else d = R.dst1 >= 0 ? R.dst1 + (code - R.ml) : -1;
    if (d < 0) continue;
    double acc = 0.0;
    for (int e = 0; e < width; ++e) {
      const long long yp = ypos[R.yidx + e];
      if (yp < 0) continue;
      acc = fma(base[R.cval + e], base[R.ybase + yp * R.ldy + c], acc);
    }
    base[d] = acc;
  }
}

// X[col] = y[col] - sum_j Y^L[col][j] s[j] - sum_j Y^U[col][j] t[j] for
// every interface unknown (one wave each): its inner solution row against
// the reduced solution of the gaps on both sides of its layer (the j-th
// coupling's column of the row at icol[C.cm + j], the right-hand side at
// column rc).
__global__ void __launch_bounds__(256) k_lsc_back(const double* __restrict__ base,
                                                  const LscCol* __restrict__ cols,
                                                  const int* __restrict__ icol, int n, int rc,
                                                  double* __restrict__ X) {
  const int wg = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int L = threadIdx.x & 63;
  if (wg >= n) return;
  const LscCol C = cols[wg];
  const double* y = base + C.xrow;
  const int* ic = icol + C.cm;
  double acc = 0.0;
  if (C.sofs >= 0)
    for (int j = L; j < C.ml; j += 64) acc = fma(y[ic[j]], base[C.sofs + j], acc);
  if (C.tofs >= 0)
    for (int j = L; j < C.mu; j += 64) acc = fma(y[ic[C.ml + j]], base[C.tofs + j], acc);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (L == 0) X[wg] = y[rc] - acc;
}

}  // namespace

namespace {
template <int TM, int TN, int KC>
hipError_t rect_launch(double* base, const BcrGemm* tasks, int ntask, const RectShape& S, hipStream_t s) {
  const long long per = (long long)(S.m / TM) * (S.n / TN);
  if ((long long)ntask * per > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * rect_lds_doubles<TM, TN, KC>();
  hipLaunchKernelGGL((k_rect_gemm<TM, TN, KC>), dim3((unsigned)(ntask * per)), dim3(256), lds, s, base,
                     tasks, S);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_rect_gemm(double* base, const BcrGemm* tasks, int ntask, const RectShape& S,
                            hipStream_t s) {
  if (ntask <= 0) return hipSuccess;
  if (S.m % 32 || S.n % 32 || S.k % 32 || S.m <= 0 || S.n <= 0 || S.k <= 0) return hipErrorInvalidValue;
  // 64 x 64 tiles where they divide the product and still give every CU two
  // workgroups (half the operand traffic per multiply-add of 32 x 32 tiles),
  // with k in chunks of 16 (17 KB of LDS: more resident workgroups per CU
  // hide more of the operand loads than longer chunks do); 32 x 32 tiles
  // otherwise.  Measured on the 3-D workload's reduced system: 128 x 128,
  // 128 x 64 and 64 x 128 tiles, chunks of 32 and 8, and 96 x 96 tiles for
  // the inner products were no faster.
  if (S.m % 64 == 0 && S.n % 64 == 0 && (long long)ntask * (S.m / 64) * (S.n / 64) >= 512)
    return rect_launch<64, 64, 16>(base, tasks, ntask, S, s);
  if (S.k % 64 == 0) return rect_launch<32, 32, 64>(base, tasks, ntask, S, s);
  return rect_launch<32, 32, 32>(base, tasks, ntask, S, s);
}

hipError_t launch_rect_gemm_win(double* base, const BcrGemm* tasks, int ntask, const RectShape& S,
                                int maxnt, hipStream_t s) {
  if (ntask <= 0) return hipSuccess;
  if (S.m % 32 || S.n % 32 || S.k % 32 || S.m <= 0 || S.n <= 0 || S.k <= 0) return hipErrorInvalidValue;
  maxnt = std::max(1, std::min(maxnt, S.n / 32));
  const long long n = (long long)ntask * (S.m / 32) * maxnt;
  if (n > 0x7fffffffLL) return hipErrorInvalidValue;
  if (S.k % 64 == 0) {
    const size_t lds = sizeof(double) * rect_lds_doubles<32, 32, 64>();
    hipLaunchKernelGGL((k_rect_gemm_win<32, 32, 64>), dim3((unsigned)n), dim3(256), lds, s, base, tasks, S,
                       maxnt);
  } else {
    const size_t lds = sizeof(double) * rect_lds_doubles<32, 32, 32>();
    hipLaunchKernelGGL((k_rect_gemm_win<32, 32, 32>), dim3((unsigned)n), dim3(256), lds, s, base, tasks, S,
                       maxnt);
  }
  return hipGetLastError();
}

namespace {
template <int TM, int TN, int KC>
hipError_t rect_launch2(double* base, const BcrGemm* ta, int na, const RectShape& SA, const BcrGemm* tb,
                        int nb, const RectShape& SB, hipStream_t s) {
  const long long n = (long long)na * (SA.m / TM) * (SA.n / TN) + (long long)nb * (SB.m / TM) * (SB.n / TN);
  if (n > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * rect_lds_doubles<TM, TN, KC>();
  hipLaunchKernelGGL((k_rect_gemm2<TM, TN, KC>), dim3((unsigned)n), dim3(256), lds, s, base, ta, na, SA, tb,
                     SB);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_rect_gemm2(double* base, const BcrGemm* ta, int na, const RectShape& SA,
                             const BcrGemm* tb, int nb, const RectShape& SB, hipStream_t s) {
  if (na <= 0) return launch_rect_gemm(base, tb, nb, SB, s);
  if (nb <= 0) return launch_rect_gemm(base, ta, na, SA, s);
  for (const RectShape* S : {&SA, &SB})
    if (S->m % 32 || S->n % 32 || S->k % 32 || S->m <= 0 || S->n <= 0 || S->k <= 0) return hipErrorInvalidValue;
  if (SA.k != SB.k) return hipErrorInvalidValue;
  const long long t64 = (long long)na * (SA.m / 64) * (SA.n / 64) + (long long)nb * (SB.m / 64) * (SB.n / 64);
  if (SA.m % 64 == 0 && SA.n % 64 == 0 && SB.m % 64 == 0 && SB.n % 64 == 0 && t64 >= 512)
    return rect_launch2<64, 64, 16>(base, ta, na, SA, tb, nb, SB, s);
  if (SA.k % 64 == 0) return rect_launch2<32, 32, 64>(base, ta, na, SA, tb, nb, SB, s);
  return rect_launch2<32, 32, 32>(base, ta, na, SA, tb, nb, SB, s);
}

hipError_t launch_fill_ones(double* base, const ZeroRun* runs, int nruns, const long long* ones,
                            long long nones, hipStream_t s) {
  for (int i = 0; i < nruns; ++i) {
    const ZeroRun& z = runs[i];
    const long long n = z.len * z.nrep;
    if (n > 0)
      hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, base + z.off,
                         z.len, z.stride, z.nrep);
  }
  if (nones > 0)
    hipLaunchKernelGGL(k_set_ones, dim3((unsigned)((nones + 255) / 256)), dim3(256), 0, s, base, ones,
                       nones);
  return hipGetLastError();
}

hipError_t launch_lsc_outer_rows(double* base, const LscRow* rows, const long long* ypos,
                                 const int* cmap, int nrow, int ncol, int width, hipStream_t s) {
  if (nrow <= 0) return hipSuccess;
  const int chunks = (ncol + 255) / 256;
  hipLaunchKernelGGL(k_lsc_outer_rows, dim3(nrow, chunks), dim3(256), 0, s, base, rows, ypos, cmap,
                     nrow, ncol, width);
  return hipGetLastError();
}

hipError_t launch_lsc_back(const double* base, const LscCol* cols, const int* icol, int n, int rc,
                           double* X, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lsc_back, dim3((n + 3) / 4), dim3(256), 0, s, base, cols, icol, n, rc, X);
  return hipGetLastError();
}

}  // namespace mrcm
