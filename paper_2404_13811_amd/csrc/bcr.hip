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
#include "pivot4.h"

#include <type_traits>

namespace mrcm {
namespace {

// ------------------------------------------------------------------ inverse
// In-place Gauss-Jordan inversion of one n x n block (n <= 128, n % 8 == 0)
// per workgroup of 512 threads; thread (tr, tc) holds the 4 x 8 tile at rows
// 4 tr.., columns 8 tc.. in registers.  Pivots are taken four at a time
// (block Gauss-Jordan without pivoting): for the pivot rows and columns K,
// with P = A[K][K],
//   A[K][j] <- P^{-1} A[K][j],   A[i][K] <- -A[i][K] P^{-1},
//   A[K][K] <- P^{-1},           A[i][j] <- A[i][j] - A[i][K] P^{-1} A[K][j],
// which equals four scalar pivot steps.  Thread 16 tr + tc holds tile
// (tr, tc), so a tile row is one row of 16 lanes of a wave.  The pivot rows
// of a step are one tile row and the pivot columns half a tile column.  One
// step, with R = P^{-1} A~[K][:] (A~ with unit vectors in the columns K)
// already in LDS:
//   1. every thread applies the rank-4 update A[i][j] <- A[i][j] -
//      A[i][K] R[:, j] to its tile (zero base in the columns K) and the
//      owners of rows K take R.  A[i][K] of a tile row is held by one lane
//      of the same 16-lane row (the owner of the pivot columns), and row
//      broadcasts hand it to the other 15: the columns never go through LDS;
//   2. look-ahead: the wave that holds the next step's pivot rows runs its
//      update at raised priority, publishes those rows to LDS, factors the
//      next 4 x 4 pivot block (closed form, redundantly in every lane) and
//      forms the next R, two columns per lane, while the other waves are
//      still updating;
//   3. one barrier.
// R alternates between two LDS buffers.  It is stored in 16-byte pieces
// interleaved over the tile columns so that the update reads are free of
// bank conflicts.  Two waves per SIMD hide each other's LDS latency.
constexpr int TR = 4, TC = 8, PB = 4;  // tile rows / columns; pivots per step
constexpr int kInvThreads = 512;

// cv[i][m] = w[i][K2 + m] of lane KT of this lane's row of 16 lanes
template <int KT, int K2>
__device__ __forceinline__ void bcast_cols(const double w[TR][TC], double cv[TR][PB]) {
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int m = 0; m < PB; ++m) {
      const long long u = __builtin_bit_cast(long long, w[i][K2 + m]);
      const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffffLL), 0x150 + KT, 0xF, 0xF, false);
      const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0x150 + KT, 0xF, 0xF, false);
      cv[i][m] = __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
    }
}

template <int K2>
__device__ __forceinline__ void bcast_cols(int kt, const double w[TR][TC], double cv[TR][PB]) {
  switch (kt) {
#define MRCM_BC(N) \
  case N:          \
    bcast_cols<N, K2>(w, cv); \
    break;
    MRCM_BC(0) MRCM_BC(1) MRCM_BC(2) MRCM_BC(3) MRCM_BC(4) MRCM_BC(5) MRCM_BC(6) MRCM_BC(7)
    MRCM_BC(8) MRCM_BC(9) MRCM_BC(10) MRCM_BC(11) MRCM_BC(12) MRCM_BC(13) MRCM_BC(14) MRCM_BC(15)
#undef MRCM_BC
    default:
      break;
  }
}

// R = P^{-1} A~[K][:] of step st (pivots K = 4 st .. 4 st + 3, A~ with
// unit vectors in the columns K), formed by the one wave that holds the
// pivot rows (tile row st): its 16 lanes of that tile row publish the rows
// to rp, then every lane of the wave forms two columns of R into rq (the
// interleaved pieces the update reads).  Returns whether the pivot block
// is unusable (zero, infinite or NaN pivot).
__device__ __forceinline__ bool form_r(int st, int t, int tr, int bp, int ntc, int c0,
                                       const double w[TR][TC], double* rp, double* rq) {
  if (tr == st) {
#pragma unroll
    for (int m = 0; m < PB; ++m) {
      double2* d = reinterpret_cast<double2*>(rp + m * kBcrInvMax + c0);
#pragma unroll
      for (int jj = 0; jj < TC / 2; ++jj) d[jj] = make_double2(w[m][2 * jj], w[m][2 * jj + 1]);
    }
  }
  // the rows are read by other lanes of the same wave: LDS stores complete
  // before the loads below
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  const int k = st * PB;
  double P[PB][PB];
#pragma unroll
  for (int m = 0; m < PB; ++m)
#pragma unroll
    for (int j = 0; j < PB; ++j) P[m][j] = rp[m * kBcrInvMax + k + j];
  const PivBlock<double> q = piv_block(P);
  const bool bad = !(piv_usable(q.d0) && piv_usable(q.da) && piv_usable(q.s0) && piv_usable(q.ds));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int col = (t & 63) + 64 * h;
    if (col < bp) {
      const int ck = col - k;
      const bool pc = ck >= 0 && ck < PB;
      double r[PB], v[PB];
      // unit vector in the pivot columns, formed arithmetically (a select
      // on a load becomes a branch with its own LDS wait)
#pragma unroll
      for (int m = 0; m < PB; ++m)
        r[m] = fma(rp[m * kBcrInvMax + col], pc ? 0.0 : 1.0, (pc && ck == m) ? 1.0 : 0.0);
      piv_apply(q, r, v);
      const int tq = col / TC, jj = (col % TC) / 2, e = col & 1;
#pragma unroll
      for (int m = 0; m < PB; ++m) rq[((m * (TC / 2) + jj) * ntc + tq) * 2 + e] = v[m];
    }
  }
  return bad;
}

__global__ void __launch_bounds__(kInvThreads) k_bcr_inv(double* __restrict__ pool,
                                                         const long long* __restrict__ offs,
                                                         const int* __restrict__ npiv, int bp,
                                                         int ld, int* flags) {
  __shared__ __align__(16) double rpan[PB * kBcrInvMax];     // [m][col] = A[k + m][col]
  __shared__ __align__(16) double rpp[2][PB * kBcrInvMax];   // R, interleaved pieces
  double* A = pool + offs[blockIdx.x];
  const int ntr = bp / TR, ntc = bp / TC;  // tiles per column / per row
  const int t = threadIdx.x;
  const int tr = t >> 4, tc = t & 15;
  const bool act = tr < ntr && tc < ntc;
  const int r0 = tr * TR, c0 = tc * TC;
  double w[TR][TC];
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TC; ++j) w[i][j] = 0.0;
  if (act) {
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      const double2* src = reinterpret_cast<const double2*>(A + (long long)(r0 + i) * ld + c0);
#pragma unroll
      for (int jj = 0; jj < TC / 2; ++jj) {
        const double2 u = src[jj];
        w[i][2 * jj] = u.x;
        w[i][2 * jj + 1] = u.y;
      }
    }
  }
  // pivots beyond the block's own size act on identity padding, which
  // they leave unchanged: skipped
  const int kend = npiv[blockIdx.x];
  const int nstep = (kend + PB - 1) / PB;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // holds tile rows 4 wv .. 4 wv + 3
  bool bad = false;
  if (nstep > 0 && wv == 0) bad |= form_r(0, t, tr, bp, ntc, c0, w, rpan, rpp[0]);
  __syncthreads();
  for (int kt = 0; kt * TC < kend; ++kt) {
    const bool own_c = tc == kt;
#pragma unroll
    for (int k2 = 0; k2 < TC; k2 += PB) {
      const int st = kt * (TC / PB) + k2 / PB;  // step: pivots 4 st .. 4 st + 3
      if (st >= nstep) break;
      const bool own_r = tr == st;
      // the wave that holds the next step's pivot rows updates first, then
      // forms that step's R while the other waves finish this update
      const bool ahead = st + 1 < nstep && wv == (st + 1) / (64 / 16);
      if (ahead) __builtin_amdgcn_s_setprio(2);
      {
        // every lane takes part in the row broadcasts
        double rv[PB][TC], cv[TR][PB];
        if (k2 == 0) bcast_cols<0>(kt, w, cv);
        else bcast_cols<PB>(kt, w, cv);
        const double2* q2 = reinterpret_cast<const double2*>(rpp[st & 1]);
#pragma unroll
        for (int m = 0; m < PB; ++m)
#pragma unroll
          for (int jj = 0; jj < TC / 2; ++jj) {
            const double2 x = q2[(m * (TC / 2) + jj) * ntc + tc];
            rv[m][2 * jj] = x.x;
            rv[m][2 * jj + 1] = x.y;
          }
        if (own_c) {
#pragma unroll
          for (int i = 0; i < TR; ++i)
#pragma unroll
            for (int m = 0; m < PB; ++m) w[i][k2 + m] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
          for (int j = 0; j < TC; ++j) {
            double acc = w[i][j];
#pragma unroll
            for (int m = 0; m < PB; ++m) acc = fma(-cv[i][m], rv[m][j], acc);
            w[i][j] = acc;
          }
        if (own_r) {
#pragma unroll
          for (int m = 0; m < PB; ++m)
#pragma unroll
            for (int j = 0; j < TC; ++j) w[m][j] = rv[m][j];
        }
      }
      if (ahead) {
        bad |= form_r(st + 1, t, tr, bp, ntc, c0, w, rpan, rpp[(st + 1) & 1]);
        __builtin_amdgcn_s_setprio(0);
      }
      __syncthreads();
    }
  }
  if (act) {
#pragma unroll
    for (int i = 0; i < TR; ++i) {
      double2* dst = reinterpret_cast<double2*>(A + (long long)(r0 + i) * ld + c0);
#pragma unroll
      for (int jj = 0; jj < TC / 2; ++jj) dst[jj] = make_double2(w[i][2 * jj], w[i][2 * jj + 1]);
    }
  }
  if (bad) atomicOr(flags, kFlagSingular);
}

// ------------------------------------------------------------------ products
// C = [C0] + al1 A1 B1 + al2 A2 B2 for a batch of tasks; the operands are
// n x n matrices at element offsets in the pool with leading dimension ld
// (whole blocks, or quarters of a block in the two-by-two inverse).  One
// workgroup of 256 threads (four waves) per 32 x 32 output tile.
constexpr int GT = 32;

typedef double dbl4 __attribute__((ext_vector_type(4)));

// One 32 x 32 output tile of a product task (tile = row-major tile index).
// Each of the four waves computes one 16 x 16 quadrant with FP64 matrix
// instructions (16 x 16 x 4 per instruction: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] of the k-slice and holds D[4r + l / 16][l % 16] in
// accumulator element r); two accumulators alternate over the k-slices so
// that consecutive instructions do not wait on each other.
//
// The k dimension of every product term is cut into chunks of KC: the A
// rows of the tile (32 x KC, row-major with stride KC + 1 so that the
// strip's rows start in different banks) and the B columns (KC x 32) of a
// chunk are staged in LDS, and the global loads of the next chunk (of this
// term or the next) are in flight while the matrix instructions run on the
// current one.  A small KC keeps the LDS of a workgroup small enough for
// several workgroups per CU.
template <int KC>
__host__ __device__ constexpr size_t gemm_lds_doubles() {
  return (size_t)GT * (KC + 1) + (size_t)KC * GT;
}

template <int KC>
__device__ __forceinline__ void gemm_tile(double* pool, const BcrGemm& T, int n, int ld, int tile,
                                          double* smem) {
  constexpr int NA = GT * KC / 256;  // A (and B) elements per thread per chunk
  constexpr int AS = KC + 1;
  double* As = smem;            // GT x (KC + 1)
  double* Bs = smem + GT * AS;  // KC x GT
  const int ntile = n / GT;
  const int tr0 = (tile / ntile) * GT, tc0 = (tile % ntile) * GT;
  const int tid = threadIdx.x;
  const int wv = tid >> 6, ln = tid & 63;
  const int qr = (wv >> 1) * 16, qc = (wv & 1) * 16;  // quadrant of this wave
  const int li = ln & 15, lk = ln >> 4;
  const int t0 = T.a1 >= 0 ? 0 : 1;  // first product term present
  const int nterm = (T.a1 >= 0 ? 1 : 0) + (T.a2 >= 0 ? 1 : 0);
  const int nch = n / KC, total = nterm * nch;
  double va[NA], vb[NA];
  auto load = [&](int c) {
    const int term = c < nch ? t0 : 1;
    const int k0 = (c % nch) * KC;
    const double* A = pool + (term ? T.a2 : T.a1);
    const double* B = pool + (term ? T.b2 : T.b1);
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = u * 256 + tid;
      const int ra = e / KC, ka = e % KC;  // A row-major: consecutive k
      const int kb = e >> 5, cb = e & 31;  // B: 32 consecutive columns
      va[u] = A[(long long)(tr0 + ra) * ld + k0 + ka];
      vb[u] = B[(long long)(k0 + kb) * ld + tc0 + cb];
    }
  };
  dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  if (total > 0) load(0);
  for (int c = 0; c < total; ++c) {
    const double al = (c < nch ? t0 : 1) ? T.al2 : T.al1;
    if (c) __syncthreads();  // the previous chunk's operands are read
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = u * 256 + tid;
      As[(e / KC) * AS + e % KC] = al * va[u];
      Bs[e] = vb[u];
    }
    __syncthreads();
    if (c + 1 < total) load(c + 1);
    const double* ap = As + (qr + li) * AS + lk;
    const double* bq = Bs + lk * GT + qc + li;
#pragma unroll
    for (int k = 0; k < KC; k += 8) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[k], bq[k * GT], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[k + 4], bq[(k + 4) * GT], acc1, 0, 0, 0);
    }
  }
  double* C = pool + T.c;
  const double* C0 = T.c0 >= 0 ? pool + T.c0 : nullptr;
  const int col = tc0 + qc + li;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const long long row = tr0 + qr + 4 * r + lk;
    double v = acc0[r] + acc1[r];
    if (C0) v += C0[row * ld + col];
    C[row * ld + col] = v;
  }
}

template <int KC>
__global__ void __launch_bounds__(256) k_bcr_gemm(double* __restrict__ pool,
                                                  const BcrGemm* __restrict__ tasks, int n, int ld) {
  extern __shared__ double smem[];
  const int ntile = n / GT;
  const int task = blockIdx.x / (ntile * ntile);
  gemm_tile<KC>(pool, tasks[task], n, ld, blockIdx.x - task * ntile * ntile, smem);
}

// y = [y0] + al1 A1 x1 + al2 A2 x2.  Workgroup (task, group of 16 rows);
// 16 lanes per row, each with bp/16 independent loads, then a 16-lane sum.
__device__ __forceinline__ void gemv_rows(const double* pool, double* __restrict__ vec, const BcrGemv& T,
                                          int bp, int rg) {
  const long long bs = (long long)bp * bp;
  const int r = rg * 16 + (threadIdx.x >> 4), l = threadIdx.x & 15;
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

__global__ void __launch_bounds__(256) k_bcr_gemv(const double* __restrict__ pool,
                                                  double* __restrict__ vec,
                                                  const BcrGemv* __restrict__ tasks, int bp) {
  gemv_rows(pool, vec, tasks[blockIdx.x], bp, blockIdx.y);
}

// Block products and block-vector products that do not depend on each
// other, in one launch: workgroups [0, ngblk) are product tiles, the rest
// row groups of the vector tasks.  The caller guarantees that no vector
// task reads a block a product task of the same launch writes.
template <int KC>
__global__ void __launch_bounds__(256) k_bcr_gemm_gemv(double* pool, double* __restrict__ vec,
                                                       const BcrGemm* __restrict__ gtasks, int ngblk,
                                                       const BcrGemv* __restrict__ vtasks, int n,
                                                       int ld, int bp) {
  extern __shared__ double smem[];
  const int b = blockIdx.x;
  if (b < ngblk) {
    const int ntile = n / GT;
    const int task = b / (ntile * ntile);
    gemm_tile<KC>(pool, gtasks[task], n, ld, b - task * ntile * ntile, smem);
  } else {
    const int rgs = bp / 16;
    const int i = b - ngblk;
    gemv_rows(pool, vec, vtasks[i / rgs], bp, i - (i / rgs) * rgs);
  }
}

// Initial state of the reduction in one pass: the 3M blocks [D | L | U] of
// the pool zero except the identity on the padded diagonal of every D
// block (rows and columns past the layer's size), and the M right-hand-side
// vectors zero.  The interface moments are then written straight into
// these blocks, none of them in the padding.
__global__ void k_bcr_init(double* __restrict__ pool, double* __restrict__ vec,
                           const int* __restrict__ lsize, int M, int bp) {
  const long long bs = (long long)bp * bp;
  const long long npool = 3LL * M * bs, nvec = (long long)M * bp;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < npool) {
    const long long k = e / bs, w = e - k * bs;
    const int r = (int)(w / bp), cc = (int)(w - (long long)r * bp);
    pool[e] = (k < M && r == cc && r >= lsize[k]) ? 1.0 : 0.0;
  } else if (e < npool + nvec) {
    vec[e - npool] = 0.0;
  }
}

// x (layer-major, padded) -> X (unknown order).
__global__ void k_bcr_gather(const double* __restrict__ xv, const int* __restrict__ col_lvl,
                             const int* __restrict__ col_loc, int n, int bp, double* __restrict__ X) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) X[c] = xv[(long long)col_lvl[c] * bp + col_loc[c]];
}

}  // namespace

hipError_t launch_bcr_inv(double* pool, const long long* offs, const int* npiv, int nblk, int n,
                          int ld, int* flags,
                          hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  if (n % TC || n > kBcrInvMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bcr_inv, dim3(nblk), dim3(kInvThreads), 0, s, pool, offs, npiv, n, ld, flags);
  return hipGetLastError();
}

// Chunk of the k dimension for products of n x n blocks: whole 128-wide
// operands when n = 128 (the latency-bound case: one round of loads per
// term), 64 for larger blocks (several workgroups per CU), else 32.
template <typename F>
hipError_t with_chunk(int n, F f) {
  if (n == 128) return f(std::integral_constant<int, 128>());
  if (n % 64 == 0) return f(std::integral_constant<int, 64>());
  return f(std::integral_constant<int, 32>());
}

template <typename KF>
hipError_t gemm_lds_attr(KF kern, size_t lds) {
  if (lds > 64 * 1024)
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

hipError_t launch_bcr_gemm(double* pool, const BcrGemm* tasks, int ntask, int n, int ld, hipStream_t s) {
  if (ntask <= 0) return hipSuccess;
  if (n % GT || n > kBcrMaxBlock) return hipErrorInvalidValue;
  const int ntile = n / GT;
  return with_chunk(n, [&](auto kc) -> hipError_t {
    constexpr int KC = decltype(kc)::value;
    const size_t lds = sizeof(double) * gemm_lds_doubles<KC>();
    hipError_t e = gemm_lds_attr(k_bcr_gemm<KC>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bcr_gemm<KC>, dim3(ntask * ntile * ntile), dim3(256), lds, s, pool, tasks, n, ld);
    return hipGetLastError();
  });
}

hipError_t launch_bcr_gemm_gemv(double* pool, double* vec, const BcrGemm* gtasks, int ngemm,
                               const BcrGemv* vtasks, int ngemv, int n, int ld, int bp,
                               hipStream_t s) {
  if (ngemm <= 0 && ngemv <= 0) return hipSuccess;
  if (n % GT || n > kBcrMaxBlock || bp % 16) return hipErrorInvalidValue;
  const int ntile = n / GT;
  const int ngblk = ngemm * ntile * ntile;
  return with_chunk(n, [&](auto kc) -> hipError_t {
    constexpr int KC = decltype(kc)::value;
    const size_t lds = sizeof(double) * gemm_lds_doubles<KC>();
    hipError_t e = gemm_lds_attr(k_bcr_gemm_gemv<KC>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bcr_gemm_gemv<KC>, dim3(ngblk + ngemv * (bp / 16)), dim3(256), lds, s, pool,
                       vec, gtasks, ngblk, vtasks, n, ld, bp);
    return hipGetLastError();
  });
}

hipError_t launch_bcr_gemv(const double* pool, double* vec, const BcrGemv* tasks, int ntask, int bp,
                           hipStream_t s) {
  if (ntask <= 0) return hipSuccess;
  if (bp % 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bcr_gemv, dim3(ntask, bp / 16), dim3(256), 0, s, pool, vec, tasks, bp);
  return hipGetLastError();
}

hipError_t launch_bcr_init(double* pool, double* vec, const int* lsize, int M, int bp, hipStream_t s) {
  const long long tot = 3LL * M * bp * bp + (long long)M * bp;
  hipLaunchKernelGGL(k_bcr_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, pool, vec, lsize,
                     M, bp);
  return hipGetLastError();
}

hipError_t launch_bcr_gather(const double* xv, const int* col_lvl, const int* col_loc, int n, int bp,
                             double* X, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bcr_gather, dim3((n + 255) / 256), dim3(256), 0, s, xv, col_lvl, col_loc, n, bp, X);
  return hipGetLastError();
}

}  // namespace mrcm
