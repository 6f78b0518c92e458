// Kernels for 3-D local problems whose plane blocks have at most 64 cells
// (boxes of up to 8 x 8 cells per plane): Steps 1-2 (factor of the
// oversampled box with the seed solves fused into its forward sweep, traces
// on Gamma_i, basis functions on Omega_i), Step 4 (particular problems),
// Step 6 (factor only) and one colour phase of the smoothing sweep
// (Steps 6-7).
//
// A box is ordered x fastest; a block is one plane of cells (same z), so
// the matrix is block tridiagonal with dense plane blocks D_j (the x and y
// couplings of the plane) and diagonal couplings between planes.  The
// factor is the sequence of block inverses W_j = S_j^{-1} of the block
// LDL^T recurrence S_j = D_j - t_{j-1} W_{j-1} t_{j-1} (t: plane couplings).
// One workgroup of NW wavefronts works on one box: lane c of wave v holds
// rows 16v .. 16v + 15 of column c of the 64 x 64 block (padded with the
// identity) in 16 registers, so a box of 64-cell planes spreads its block
// over four waves (four SIMDs) and smaller planes take fewer.  W_j is
// computed in place by Gauss-Jordan elimination with four pivots per step:
// the wave holding the pivot rows publishes them through LDS, and every
// lane applies the rank-4 update to its 16 entries.  The inverses are
// symmetric, so lane c also holds entries 16v .. 16v + 15 of row c, and a
// block-vector product y = W_j z is a 16-term partial dot product per lane
// (z read from LDS) summed over the waves through LDS.  Solves:
//   forward   z_j = W_j (b_j + t_{j-1} .* z_{j-1})
//   backward  x_j = z_j + W_j (t_j .* x_{j+1}).
// The inverses are stored whole (nb x nb, row-major), the layout the
// smoothing kernel reads back.
#include "local3_common.h"
#include "pivot4.h"

namespace mrcm {
namespace {

// Pivot data of one elimination step (two alternating buffers) and the
// flag.  vb holds the step's multipliers v_c = P^-1 A[k..k+3][c] of every
// column c (m-major: lane c reads vb[m][c], no bank conflicts), rs the
// pivot-column entries A[i][k+m] of every row i (row-major, read as
// broadcasts), pb the 4 x 4 pivot block on its way to the wave that factors
// it.  vb and rs also hold the per-wave partial sums of the block-vector
// products (4 right-hand sides x NW waves x 64 lanes <= 1024 values), which
// never overlap an elimination.
struct __align__(16) Gj3 {
  double vb[2][G3 * P3];
  double rs[2][P3 * G3];
  double pb[2][G3 * G3];
  int flag;
};

__device__ __forceinline__ double* partials3(Gj3& sm) { return &sm.vb[0][0]; }

// S_j = D_j - t_{j-1} W_{j-1} t_{j-1} (the lane's 16 entries of column c),
// w holding W_{j-1} on entry when j > 0; identity outside the nb x nb block.
__device__ __forceinline__ void build3(const Geo& g, const Box& B, const Box3& s, int j, double w[R3]) {
  const int c = lane3();
  const int r0 = R3 * wave3();
  const int nb = s.m0 * s.m1, m0 = s.m0;
  const bool cin = c < nb;
  const int cc = cin ? c : 0;
  const double dc = s.Dg[j * nb + cc];
  const double txm = (cin && cc % m0 > 0) ? tplane(g, B, s, j, cc - 1, 0) : 0.0;
  const double txp = cin ? tplane(g, B, s, j, cc, 0) : 0.0;
  const double tym = (cin && cc >= m0) ? tplane(g, B, s, j, cc - m0, 1) : 0.0;
  const double typ = cin ? tplane(g, B, s, j, cc, 1) : 0.0;
  const double* tp = s.Tz + (j > 0 ? j - 1 : 0) * nb;
  const double tcp = (j > 0 && cin) ? tp[cc] : 0.0;
#pragma unroll
  for (int ii = 0; ii < R3; ++ii) {
    const int i = r0 + ii;
    // sums of selects: with one-cell-wide planes (m0 = 1) the x and y
    // neighbours of the block numbering coincide
    double v = (i == c) ? dc : 0.0;
    v -= (i == c - 1) ? txm : 0.0;
    v -= (i == c + 1) ? txp : 0.0;
    v -= (i == c - m0) ? tym : 0.0;
    v -= (i == c + m0) ? typ : 0.0;
    if (j > 0 && i < nb) v = fma(-tp[i] * tcp, w[ii], v);
    w[ii] = (i < nb && cin) ? v : (i == c ? 1.0 : 0.0);
  }
}

// In-place Gauss-Jordan inverse of the block, four pivots per step, no
// pivoting (the Schur complements are SPD).  The pivot columns are not
// exchanged: for a symmetric matrix under in-place Gauss-Jordan, column
// k + m equals row k + m on the rows not yet eliminated and its negative
// on the rows already eliminated (i < k), so the wave holding rows
// k .. k + 3 publishes them with that sign as the pivot-column entries of
// every row.  That wave also factors the 4 x 4 pivot block (closed form)
// and publishes the multipliers v_c = P^-1 A[k..k+3][c] of every column c
// (a unit right-hand side for the pivot columns), so the other waves only
// read v_c and apply the rank-4 update A[i][c] -= sum_m A[i][k+m] v_c[m] to
// their rows.  Look-ahead: during step k the wave holding rows k + 4 ..
// k + 7 updates those rows first and publishes step k + 4's pivot data
// before updating the rest, so one workgroup barrier per step suffices and
// the pivot factorisation overlaps the other waves' updates.  The step
// index is a template parameter: every register index is a compile-time
// constant.
template <int NW, int K>
__device__ __forceinline__ void gj3_pivot(int nb, Gj3& sm, double w[R3], bool& bad) {
  // publish step K's pivot data (the calling wave holds rows K .. K + 3)
  constexpr int RI = K % R3;
  const int c = lane3_here();
  const int ck = c - K;
  const bool pc = ck >= 0 && ck < G3;
  double* vb = sm.vb[(K / G3) & 1];
  double* rs = sm.rs[(K / G3) & 1];
  double* pb = sm.pb[(K / G3) & 1];
  if (pc) {
    *reinterpret_cast<double2*>(pb + ck * G3) = make_double2(w[RI], w[RI + 1]);
    *reinterpret_cast<double2*>(pb + ck * G3 + 2) = make_double2(w[RI + 2], w[RI + 3]);
  }
  const double sg = c < K ? -1.0 : 1.0;
  *reinterpret_cast<double2*>(rs + c * G3) = make_double2(sg * w[RI], sg * w[RI + 1]);
  *reinterpret_cast<double2*>(rs + c * G3 + 2) = make_double2(sg * w[RI + 2], sg * w[RI + 3]);
  bsync<1>();  // the pivot block is read back by this wave only
  double P[G3][G3], r[G3], v[G3];
#pragma unroll
  for (int j = 0; j < G3; ++j)
#pragma unroll
    for (int m = 0; m < G3; ++m) P[m][j] = pb[j * G3 + m];
#pragma unroll
  for (int m = 0; m < G3; ++m) {
    // select values, not addresses (a select between the address of a
    // constant and of w[] would keep w out of registers)
    const double wm = w[RI + m];
    const double unit = ck == m ? 1.0 : 0.0;
    r[m] = pc ? unit : wm;
  }
  const PivBlock<double> q = piv_block(P);
  bad |= !(q.d0 > 0.0 && q.da > 0.0 && q.s0 > 0.0 && q.ds > 0.0);
  piv_apply(q, r, v);
#pragma unroll
  for (int m = 0; m < G3; ++m) vb[m * P3 + c] = v[m];
  (void)nb;
}

// rows [R0, R1) of the lane's 16: A[i][c] = (pivot column ? 0 : A[i][c]) -
// sum_m rs[i][m] v[m]
template <int R0, int R1>
__device__ __forceinline__ void gj3_rows(const double* rw, unsigned long long keep, const double v[G3],
                                         double w[R3]) {
#pragma unroll
  for (int ii = R0; ii < R1; ++ii) {
    const double2 c01 = *reinterpret_cast<const double2*>(rw + ii * G3);
    const double2 c23 = *reinterpret_cast<const double2*>(rw + ii * G3 + 2);
    double acc = __longlong_as_double(__double_as_longlong(w[ii]) & keep);
    acc = fma(-c01.x, v[0], acc);
    acc = fma(-c01.y, v[1], acc);
    acc = fma(-c23.x, v[2], acc);
    acc = fma(-c23.y, v[3], acc);
    w[ii] = acc;
  }
}

template <int NW, int K>
__device__ __forceinline__ void gj3_step(int nb, Gj3& sm, double w[R3], bool& bad) {
  constexpr int OWN = K / R3, RI = K % R3;
  constexpr int KN = K + G3, OWNN = KN / R3, RIN = KN % R3;
  const int c = lane3_here();
  const int wv = wave3();
  const double* vb = sm.vb[(K / G3) & 1];
  const double* rw = sm.rs[(K / G3) & 1] + R3 * wv * G3;
  const int ck = c - K;
  const bool pc = ck >= 0 && ck < G3;
  // the pivot columns start from zero: a bit mask, not a branch per row
  const unsigned long long keep = pc ? 0ull : ~0ull;
  double v[G3];
#pragma unroll
  for (int m = 0; m < G3; ++m) v[m] = vb[m * P3 + c];
  if constexpr (KN < R3 * NW) {
    // look-ahead: every wave updates the rows at the next pivot rows' place
    // first (the order of the rows does not matter otherwise); the wave
    // that holds them then publishes the next step's pivot data before it
    // updates the rest
    gj3_rows<RIN, RIN + G3>(rw, keep, v, w);
    if (KN < nb && wv == OWNN) gj3_pivot<NW, KN>(nb, sm, w, bad);
    gj3_rows<0, RIN>(rw, keep, v, w);
    gj3_rows<RIN + G3, R3>(rw, keep, v, w);
  } else {
    gj3_rows<0, R3>(rw, keep, v, w);
  }
  if (wv == OWN) {
#pragma unroll
    for (int m = 0; m < G3; ++m) w[RI + m] = v[m];
  }
  bsync<NW>();
}

template <int NW, int K>
__device__ __forceinline__ void gj3_steps(int nb, Gj3& sm, double w[R3], bool& bad) {
  if constexpr (K < R3 * NW) {
    if (K < nb) {
      gj3_step<NW, K>(nb, sm, w, bad);
      gj3_steps<NW, K + G3>(nb, sm, w, bad);
    }
  }
}

template <int NW>
__device__ __forceinline__ void gj3(int nb, Gj3& sm, double w[R3]) {
  bool bad = false;
  if (wave3() == 0) gj3_pivot<NW, 0>(nb, sm, w, bad);
  bsync<NW>();
  gj3_steps<NW, 0>(nb, sm, w, bad);
  if (bad && lane3() == 0) atomicOr(&sm.flag, kFlagNotPD);
  bsync<NW>();
}

// The lane's share of y = W z for the staged vector z (64 values in LDS):
// the 16-term partial dot product of its entries of row c with z.
__device__ __forceinline__ double wdot3(const double w[R3], const double* z) {
  const double* zw = z + R3 * wave3();
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int ii = 0; ii < R3; ii += 2) {
    const double2 zz = *reinterpret_cast<const double2*>(zw + ii);
    a0 = fma(w[ii], zz.x, a0);
    a1 = fma(w[ii + 1], zz.y, a1);
  }
  return a0 + a1;
}

// Y[k][c] (+)= (W Z_k)[c] for the nrhs vectors staged in Z (k-th at Z + 64k),
// Y[k] at Y + k * ystride; the partial sums of the waves are added through
// LDS in a fixed order, four right-hand sides at a time.
template <int NW, bool ACC>
__device__ __forceinline__ void wmul3(const Box3& s, Gj3& sm, int nb, int nrhs, const double w[R3],
                                      double* Y, int ystride) {
  constexpr int NT = 64 * NW;
  const int c = lane3();
  if constexpr (NW == 1) {
    for (int k = 0; k < nrhs; ++k) {
      const double y = wdot3(w, s.Z + k * P3);
      if (c < nb) {
        if (ACC) Y[k * ystride + c] += y;
        else Y[k * ystride + c] = y;
      }
    }
    lsync<NW>();
  } else {
    double* pt = partials3(sm);
    const int wv = wave3();
    for (int k0 = 0; k0 < nrhs; k0 += 4) {
      const int cnt = min(4, nrhs - k0);
      for (int kk = 0; kk < cnt; ++kk) pt[(kk * NW + wv) * P3 + c] = wdot3(w, s.Z + (k0 + kk) * P3);
      lsync<NW>();
      for (int e = threadIdx.x; e < cnt * P3; e += NT) {
        const int kk = e / P3, L = e % P3;
        double y = 0.0;
#pragma unroll
        for (int u = 0; u < NW; ++u) y += pt[(kk * NW + u) * P3 + L];
        if (L < nb) {
          if (ACC) Y[(k0 + kk) * ystride + L] += y;
          else Y[(k0 + kk) * ystride + L] = y;
        }
      }
      lsync<NW>();
    }
  }
}

// Forward step of block j for all right-hand sides (W_j in w).
template <int NW>
__device__ __forceinline__ void fwd3(const Box3& s, Gj3& sm, int nb, int j, int nrhs, const double w[R3]) {
  constexpr int NT = 64 * NW;
  for (int e = threadIdx.x; e < nrhs * P3; e += NT) {
    const int k = e / P3, L = e % P3;
    double v = 0.0;
    if (L < nb) {
      v = s.X[k * s.nc + j * nb + L];
      if (j > 0) v = fma(s.Tz[(j - 1) * nb + L], s.X[k * s.nc + (j - 1) * nb + L], v);
    }
    s.Z[k * P3 + L] = v;
  }
  lsync<NW>();
  wmul3<NW, false>(s, sm, nb, nrhs, w, s.X + j * nb, s.nc);
}

// Backward step of block j (W_j in w): x_j += W_j (t_j .* x_{j+1}).
template <int NW>
__device__ __forceinline__ void bwd3(const Box3& s, Gj3& sm, int nb, int j, int nrhs, const double w[R3]) {
  constexpr int NT = 64 * NW;
  for (int e = threadIdx.x; e < nrhs * P3; e += NT) {
    const int k = e / P3, L = e % P3;
    s.Z[k * P3 + L] = L < nb ? s.Tz[j * nb + L] * s.X[k * s.nc + (j + 1) * nb + L] : 0.0;
  }
  lsync<NW>();
  wmul3<NW, true>(s, sm, nb, nrhs, w, s.X + j * nb, s.nc);
}

// The lane's entries of the cached symmetric inverse W_j (rows 16v .. of
// column c; coalesced along the rows).
__device__ __forceinline__ void load3(const double* Wj, int nb, double w[R3]) {
  const int c = lane3(), r0 = R3 * wave3();
#pragma unroll
  for (int ii = 0; ii < R3; ++ii) {
    const int i = r0 + ii;
    w[ii] = (i < nb && c < nb) ? Wj[i * nb + c] : (i == c ? 1.0 : 0.0);
  }
}

__device__ __forceinline__ void store3(double* Wj, int nb, const double w[R3]) {
  const int c = lane3(), r0 = R3 * wave3();
#pragma unroll
  for (int ii = 0; ii < R3; ++ii) {
    const int i = r0 + ii;
    if (i < nb && c < nb) Wj[i * nb + c] = w[ii];
  }
}

// Factor of the box fused with the forward sweep of nrhs right-hand sides
// already in X; inverses to Wg.
template <int NW>
__device__ __forceinline__ void factor3(const Geo& g, const Box& B, const Box3& s, double* Wg, int nrhs,
                                        Gj3& sm) {
  const int nb = s.m0 * s.m1;
  double w[R3];
#pragma unroll
  for (int i = 0; i < R3; ++i) w[i] = 0.0;
  for (int j = 0; j < s.m2; ++j) {
    build3(g, B, s, j, w);
    gj3<NW>(nb, sm, w);
    store3(Wg + (long long)j * nb * nb, nb, w);
    if (nrhs > 0) fwd3<NW>(s, sm, nb, j, nrhs, w);
  }
}

// PF: the next plane's inverse is loaded while the current one is applied
template <int NW, bool PF>
__device__ __forceinline__ void backward3(const Box3& s, Gj3& sm, const double* Wg, int nrhs) {
  const int nb = s.m0 * s.m1;
  double w[R3], wn[R3];
  if (PF && s.m2 >= 2) load3(Wg + (long long)(s.m2 - 2) * nb * nb, nb, w);
  for (int j = s.m2 - 2; j >= 0; --j) {
    if (!PF) load3(Wg + (long long)j * nb * nb, nb, w);
    if (PF && j > 0) load3(Wg + (long long)(j - 1) * nb * nb, nb, wn);
    bwd3<NW>(s, sm, nb, j, nrhs, w);
    if (PF) {
#pragma unroll
      for (int ii = 0; ii < R3; ++ii) w[ii] = wn[ii];
    }
  }
}

// Steps 1-2 on an oversampled box (FO: Step 6, the factor alone).
template <int NW, bool FO, bool TS>
__device__ __forceinline__ void basis3(const Geo& g, const Box& B, const Seed* __restrict__ seeds,
                                       const double* __restrict__ logK, double beta,
                                       double* __restrict__ fac, double* __restrict__ Pk,
                                       double* __restrict__ tr_u, double* __restrict__ tr_phi,
                                       double* __restrict__ tr_beta, double* dsm, Gj3& sm) {
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x;
  const int nrhs = FO ? 0 : B.nrhs;
  Box3 s = carve3<TS>(dsm, B, nrhs, g.kc);
  load_box3<NW, true>(g, B, logK, beta, s);
  for (int e = tid; e < nrhs * s.nc; e += NT) s.X[e] = 0.0;
  bsync<NW>();
  seed_rhs3<NW>(g, B, s, seeds, beta, nrhs, s.X);
  bsync<NW>();
  double* Wg = fac + B.fac;
  factor3<NW>(g, B, s, Wg, nrhs, sm);
  if (FO) return;
  backward3<NW, true>(s, sm, Wg, nrhs);
  basis_out3<NW>(g, B, s, seeds, beta, nrhs, Pk, tr_u, tr_phi, tr_beta);
}

// Step 4 on a subdomain: K = exp(log K) of its cells (the subdomains cover
// the grid once; a K that is not finite and positive is flagged).
template <int NW, bool TS>
__device__ __forceinline__ void particular3(const Geo& g, const Box& B,
                                            const double* __restrict__ logK, double* __restrict__ K,
                                            const double* __restrict__ f,
                                            const double* __restrict__ bcv, double beta,
                                            double* __restrict__ fac, double* __restrict__ pbar,
                                            double* __restrict__ ubar, double* __restrict__ pibar,
                                            double* dsm, Gj3& sm) {
  Box3 s = carve3<TS>(dsm, B, 1, g.kc);
  load_box3<NW, true>(g, B, logK, beta, s);
  part_k3<NW, TS>(g, B, s, K, sm.flag);
  physical3<NW>(g, B, s, f, bcv, s.X);
  bsync<NW>();
  double* Wg = fac + B.fac;
  factor3<NW>(g, B, s, Wg, 1, sm);
  backward3<NW, true>(s, sm, Wg, 1);
  part_out3<NW>(g, B, s, beta, pbar, ubar, pibar);
}

// Steps 6-7 for one box: right-hand side from the state, solve with the
// cached inverses, p on Omega_i and Omega_i's Gamma fluxes.
template <int NW, bool TS>
__device__ __forceinline__ void smooth3(const Geo& g, const Box& B, const double* __restrict__ K,
                                        const double* __restrict__ f,
                                        const double* __restrict__ bcv, double beta,
                                        const double* __restrict__ fac, double* p, double* gflux,
                                        double* dsm, Gj3& sm) {
  Box3 s = carve3<TS>(dsm, B, 1, g.kc);
  load_box3<NW, false>(g, B, K, beta, s);
  physical3<NW>(g, B, s, f, bcv, s.X);
  bsync<NW>();
  smooth_rhs3<NW>(g, B, s, p, gflux, beta, s.X);
  bsync<NW>();
  const int nb = s.m0 * s.m1;
  const double* Wg = fac + B.fac;
  double w[R3];
  for (int j = 0; j < s.m2; ++j) {
    load3(Wg + (long long)j * nb * nb, nb, w);
    fwd3<NW>(s, sm, nb, j, 1, w);
  }
  backward3<NW, false>(s, sm, Wg, 1);
  smooth_out3<NW>(g, B, s, p, gflux, beta);
}

// Register budget for three resident boxes per CU (their LDS allows no
// more): at most 168 registers per lane.
template <int NW, bool TS>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3))) k_basis3(Geo g, const Box* __restrict__ boxes,
                                                    const Seed* __restrict__ seeds,
                                                    const double* __restrict__ logK, double beta,
                                                    double* __restrict__ fac, double* __restrict__ Pk,
                                                    double* __restrict__ tr_u,
                                                    double* __restrict__ tr_phi,
                                                    double* __restrict__ tr_beta, int factor_only,
                                                    int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ Gj3 sm;
  if (threadIdx.x == 0) sm.flag = 0;
  bsync<NW>();
  const Box B = boxes[blockIdx.x];
  if (factor_only)
    basis3<NW, true, TS>(g, B, seeds, logK, beta, fac, Pk, tr_u, tr_phi, tr_beta, dsm, sm);
  else
    basis3<NW, false, TS>(g, B, seeds, logK, beta, fac, Pk, tr_u, tr_phi, tr_beta, dsm, sm);
  bsync<NW>();
  if (threadIdx.x == 0 && sm.flag) atomicOr(flags, sm.flag);
}

template <int NW, bool TS>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3))) k_particular3(Geo g, const Box* __restrict__ boxes,
                                                         const double* __restrict__ logK,
                                                         double* __restrict__ K,
                                                         const double* __restrict__ f,
                                                         const double* __restrict__ bcv, double beta,
                                                         double* __restrict__ fac,
                                                         double* __restrict__ pbar,
                                                         double* __restrict__ ubar,
                                                         double* __restrict__ pibar, int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ Gj3 sm;
  if (threadIdx.x == 0) sm.flag = 0;
  bsync<NW>();
  const Box B = boxes[blockIdx.x];
  particular3<NW, TS>(g, B, logK, K, f, bcv, beta, fac, pbar, ubar, pibar, dsm, sm);
  bsync<NW>();
  if (threadIdx.x == 0 && sm.flag) atomicOr(flags, sm.flag);
}

template <int NW, bool TS>
__global__ void __launch_bounds__(64 * NW) k_smooth3(Geo g, const Box* __restrict__ boxes,
                                                     const double* __restrict__ K,
                                                     const double* __restrict__ f,
                                                     const double* __restrict__ bcv, double beta,
                                                     const double* __restrict__ fac,
                                                     double* __restrict__ p, double* __restrict__ gflux) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ Gj3 sm;
  const Box B = boxes[blockIdx.x];
  smooth3<NW, TS>(g, B, K, f, bcv, beta, fac, p, gflux, dsm, sm);
}

template <typename KF>
hipError_t lds_attr3(KF kern, size_t bytes) {
  if (bytes > 64 * 1024)
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return hipSuccess;
}

}  // namespace

size_t box3_lds_bytes(int m0, int m1, int m2, int nrhs, int kc) {
  return sizeof(double) * box3_doubles(m0, m1, m2, nrhs, kc);
}

int box3_waves(int nb) { return nb <= R3 ? 1 : nb <= 2 * R3 ? 2 : 4; }

// waves per box, and the scalar or the tensor form of K
#define MRCM_NW_SWITCH(nw, CALL)                   \
  if (g.kc > 1) {                                  \
    switch (nw) {                                  \
      case 1: CALL(1, true); break;                \
      case 2: CALL(2, true); break;                \
      case 4: CALL(4, true); break;                \
      default: return hipErrorInvalidValue;        \
    }                                              \
  } else {                                         \
    switch (nw) {                                  \
      case 1: CALL(1, false); break;               \
      case 2: CALL(2, false); break;               \
      case 4: CALL(4, false); break;               \
      default: return hipErrorInvalidValue;        \
    }                                              \
  }

hipError_t launch_basis3(const Geo& g, const Box* boxes, int nbox, const Seed* seeds,
                         const double* logK, double beta, double* fac, double* Pk, double* tr_u,
                         double* tr_phi, double* tr_beta, int factor_only, int* flags, size_t lds,
                         int nw, hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
#define MRCM_CALL(NW, TS)                                                                             \
  e = lds_attr3(k_basis3<NW, TS>, lds);                                                               \
  if (e != hipSuccess) return e;                                                                      \
  hipLaunchKernelGGL((k_basis3<NW, TS>), dim3(nbox), dim3(64 * NW), lds, s, g, boxes, seeds, logK, beta, fac, \
                     Pk, tr_u, tr_phi, tr_beta, factor_only, flags)
  MRCM_NW_SWITCH(nw, MRCM_CALL)
#undef MRCM_CALL
  return hipGetLastError();
}

hipError_t launch_particular3(const Geo& g, const Box* boxes, int nbox, const double* logK, double* K,
                              const double* f, const double* bcv, double beta, double* fac,
                              double* pbar, double* ubar, double* pibar, int* flags, size_t lds, int nw,
                              hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
#define MRCM_CALL(NW, TS)                                                                            \
  e = lds_attr3(k_particular3<NW, TS>, lds);                                                         \
  if (e != hipSuccess) return e;                                                                     \
  hipLaunchKernelGGL((k_particular3<NW, TS>), dim3(nbox), dim3(64 * NW), lds, s, g, boxes, logK, K, f, bcv, \
                     beta, fac, pbar, ubar, pibar, flags)
  MRCM_NW_SWITCH(nw, MRCM_CALL)
#undef MRCM_CALL
  return hipGetLastError();
}

hipError_t launch_smooth3(const Geo& g, const Box* boxes, int nmem, const double* K, const double* f,
                          const double* bcv, double beta, const double* fac, double* p, double* gflux,
                          size_t lds, int nw, hipStream_t s) {
  if (nmem <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
#define MRCM_CALL(NW, TS)                                                                               \
  e = lds_attr3(k_smooth3<NW, TS>, lds);                                                                \
  if (e != hipSuccess) return e;                                                                        \
  hipLaunchKernelGGL((k_smooth3<NW, TS>), dim3(nmem), dim3(64 * NW), lds, s, g, boxes, K, f, bcv, beta, fac, p, \
                     gflux)
  MRCM_NW_SWITCH(nw, MRCM_CALL)
#undef MRCM_CALL
  return hipGetLastError();
}

#undef MRCM_NW_SWITCH

}  // namespace mrcm
