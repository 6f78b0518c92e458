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

#include <hip/hip_cooperative_groups.h>

#include <algorithm>

namespace mrcm {
namespace {

using namespace wave;




// Store the nb x nb block held in the register layout w to Wj.
__device__ __forceinline__ void store_block(int nb, double* Wj, const double w[HB]) {
  // lower triangle, row-major (the layout block_src reads)
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
#pragma unroll
  for (int i = 0; i < HB; ++i) {
    const int r = HB * h + i;
    if (r < nb && c <= r) Wj[r * (r + 1) / 2 + c] = w[i];
  }
}

// Block j of the cached FP64 factors of a box
__device__ __forceinline__ double* fblock(double* Wg, int nb, int j) {
  return Wg + (long long)j * block_elems<double>(nb);
}

// Factorisation fused with the forward sweep; inverses to Wg, couplings to Tg.
__device__ __forceinline__ void factor_forward(const Box& B, double* Wg, double* Tg, int nrhs, const BoxLds& s,
                               WaveSmem& sm) {
  const int L = lane_id();
  const int nb = B.nb;
  for (int e = L; e < B.ncell; e += 64) Tg[e] = s.Tn[e];
  double w[HB];
#pragma unroll
  for (int i = 0; i < HB; ++i) w[i] = 0.0;
  for (int j = 0; j < B.nblk; ++j) {
    wbuild(nb, j, s, w);
    wgj(nb, sm, w);
    store_block(nb, fblock(Wg, nb, j), w);
    fwd_step(nb, B.ncell, j, nrhs, s, w);
  }
}


// ------------------------------------------------------------------ kernels

// LDS of a basis box: the box arrays with its right-hand sides (the Z
// scratch of BoxLds serves wave 0), the Z scratch of wave 1, and the forward
// Schur complement of the meeting block (nb x nb, nb = m0, row-major).
__host__ __device__ inline size_t basis_lds_doubles(int m0, int m1, int nrhs, int kc = 1) {
  return box_lds_doubles(m0, m1, nrhs, kc) + (size_t)nrhs * NBW + (size_t)m0 * m0 + 2;
}

// Steps 1-2: factor the oversampled box, solve every seed, extract
// u and phi on Gamma_i and the restriction to Omega_i.  Two waves solve
// the block-tridiagonal system from both ends (meeting block m = nblk / 2):
// wave 0 eliminates blocks 0 .. m-1 (forward inverses W_j into fac), wave 1
// blocks nblk-1 .. m+1 (backward inverses W'_j = (D_j - t_j W'_{j+1} t_j)^{-1}
// into fact), each with the forward sweep of every seed fused in; wave 1
// then inverts Z_m = (S_m - t_m W'_{m+1} t_m)^{-1} (S_m: forward Schur
// complement of block m, from wave 0), stored at block m of fact, and solves
// the meeting block; both back-substitute outwards.  The chain of block
// inverses on one wave is about half as long as a one-ended elimination,
// and fac / fact are exactly the factors of the two-ended smoothing sweep.
// FO (factor only, Algorithm 1 Step 6): the box is factored with the
// smoothing Robin parameter and nothing else is solved or written (the
// block couplings do not depend on beta and are shared with Step 1).
template <bool FO = false>
__device__ __forceinline__ void basis_box(const Geo& g, const Box& B, const Seed* __restrict__ seeds,
                                          const double* __restrict__ logK, double beta,
                                          double* __restrict__ fac, double* __restrict__ fact,
                                          double* __restrict__ tcoup,
                                          double* __restrict__ Pk, double* __restrict__ tr_u,
                                          double* __restrict__ tr_phi,
                                          double* __restrict__ tr_beta, double* dsm, WaveSmem* sm) {
  const int L = lane_id();
  const int tid = threadIdx.x, wv = tid >> 6;
  const int nrhs = FO ? 0 : B.nrhs;
  BoxLds s = carve(dsm, B, nrhs, g.kc);
  double* Z1 = s.Z + nrhs * NBW;
  double* Sm = Z1 + nrhs * NBW;
  const int nc = B.ncell;
  // set-up by both waves: box arrays (K from log K), seed right-hand
  // sides, couplings
  load_box<128, true>(g, B, logK, beta, s);
  for (int e = tid; e < nrhs * nc; e += 128) s.X[e] = 0.0;
  __syncthreads();
  // T^R times the seed on the cells of its side, all seeds at once
  const int fs = s.m0 > s.m1 ? s.m0 : s.m1;  // faces of the longest side
  #pragma unroll 1
  for (int e = tid; e < nrhs * fs; e += 128) {
    const int k = e / fs, t = e % fs;
    const Seed sd = seeds[B.seed0 + k];
    const int a = sd.side >> 1, so = sd.side & 1;
    const int nf = (a == 0) ? s.m1 : s.m0;
    if (t >= nf) continue;
    int c[3];
    if (a == 0) { c[0] = so ? B.hi[0] - 1 : B.lo[0]; c[1] = B.lo[1] + t; }
    else { c[1] = so ? B.hi[1] - 1 : B.lo[1]; c[0] = B.lo[0] + t; }
    c[2] = 0;
    const int ox = c[0] + (a == 0 ? (so ? 1 : -1) : 0), oy = c[1] + (a == 1 ? (so ? 1 : -1) : 0);
    const double kc = kat(s, B, c[0], c[1], a);
    const double bt = robin_beta(g, a, kc, kat(s, B, ox, oy, a), beta);
    s.X[k * nc + bloc(B, s, c[0], c[1])] = robin_T(g, kc, bt) * seed_value(g, sd, B.lo, B.hi, c);
  }
  if (!FO)
    for (int e = tid; e < nc; e += 128) tcoup[B.scr + e] = s.Tn[e];
  __syncthreads();
  const int nb = B.nb, nblk = B.nblk, m = nblk / 2;
  double* Wf = fac + B.fac;
  double* Wt = fact + B.fac;
  double w[HB];
#pragma unroll
  for (int i = 0; i < HB; ++i) w[i] = 0.0;
  if (wv == 0) {
    for (int j = 0; j < m; ++j) {
      wbuild(nb, j, s, w);
      wgj(nb, sm[0], w);
      store_block(nb, fblock(Wf, nb, j), w);
      fwd_step_d(nb, nc, j, j - 1, j > 0, nrhs, s, s.Z, w);
    }
    wbuild(nb, m, s, w);  // S_m
    const int c = L & 31, h = L >> 5;
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const int r = HB * h + i;
      if (r < nb && c < nb) Sm[r * nb + c] = w[i];
    }
  } else {
    for (int j = nblk - 1; j > m; --j) {
      wbuild_t(nb, j, j < nblk - 1 ? j : -1, s, w);
      wgj(nb, sm[1], w);
      store_block(nb, fblock(Wt, nb, j), w);
      fwd_step_d(nb, nc, j, j + 1, j < nblk - 1, nrhs, s, Z1, w);
    }
  }
  __syncthreads();
  if (wv == 1) {
    // Z_m = (S_m - t_m W'_{m+1} t_m)^{-1}, identity padding kept; w holds
    // W'_{m+1} when the bottom half is not empty
    const int c = L & 31, h = L >> 5;
    const double* Tm = s.Tn + m * nb;
    const double tc = (m < nblk - 1 && c < nb) ? Tm[c] : 0.0;
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const int r = HB * h + i;
      // identity padding outside the nb x nb block, as wbuild leaves it
      const double smi = (r < nb && c < nb) ? Sm[r * nb + c] : (r == c ? 1.0 : 0.0);
      const double tr = (m < nblk - 1 && r < nb) ? Tm[r] : 0.0;
      w[i] = (m < nblk - 1 && r < nb && c < nb) ? fma(-tr * tc, w[i], smi) : smi;
    }
    wgj(nb, sm[1], w);
    store_block(nb, fblock(Wt, nb, m), w);
    if (!FO) mid_step(nb, nc, m, nblk, nrhs, s, Z1, w);
  }
  if (FO) return;
  __syncthreads();
  if (wv == 0) twist_back_cached(B, Wf, nrhs, s, s.Z, false);
  else twist_back_cached(B, Wt, nrhs, s, Z1, true);
  __syncthreads();
  int olo[3], ohi[3];
  womega(g, B.sub, olo, ohi);
  const int ncell_o = g.S[0] * g.S[1];
  #pragma unroll 1
  for (int e = tid; e < nrhs * ncell_o; e += 128) {
    const int k = e / ncell_o, t = e % ncell_o;
    Pk[(long long)(B.seed0 + k) * ncell_o + t] =
        s.X[k * nc + bloc(B, s, olo[0] + t % g.S[0], olo[1] + t / g.S[0])];
  }
  for (int q = 0; q < 4; ++q) {
    const int nf = (q >> 1) == 0 ? g.S[1] : g.S[0];
    const bool has = wneighbor(g, B.sub, q) >= 0;
    const int a = q >> 1, so = q & 1;
    #pragma unroll 1
    for (int e = tid; e < nrhs * nf; e += 128) {
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

// Step 4: particular problem on Omega_i with zero Robin data on Gamma_i.
// The box is Omega_i itself: it also writes K = exp(log K) of its cells
// (the subdomains cover the grid once) and flags a K that is not finite
// and positive.
__device__ __forceinline__ void particular_box(const Geo& g, const Box& B,
                                               const double* __restrict__ logK,
                                               double* __restrict__ K,
                                               const double* __restrict__ f,
                                               const double* __restrict__ bcv, double beta,
                                               double* __restrict__ fac, double* __restrict__ tcoup,
                                               double* __restrict__ pbar, double* __restrict__ ubar,
                                               double* __restrict__ pibar, double* dsm, WaveSmem& sm) {
  const int L = lane_id();
  BoxLds s = carve(dsm, B, 1, g.kc);
  load_box<64, true>(g, B, logK, beta, s);
  for (int t = L; t < B.ncell; t += 64) {
    const int x = B.lo[0] + t % s.m0, y = B.lo[1] + t / s.m0;
    for (int a = 0; a < g.kc; ++a) {
      const double k = kat(s, B, x, y, a);
      if (!(k > 0.0) || !isfinite(k)) atomicOr(&sm.flag, kFlagBadK);
      K[kaxis(g, a) + x + g.n[0] * y] = k;
    }
  }
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
      const double kc = kat(s, B, x, y, a);
      const double bt = robin_beta(g, a, kc, kat(s, B, ox, oy, a), beta);
      const double u = robin_T(g, kc, bt) * s.X[bloc(B, s, x, y)] / g.area;
      ubar[oidx] = u;
      pibar[oidx] = bt * u;
    }
  }
}

// Steps 1-2 and 4 in one launch of two-wave workgroups.  Workgroups
// [0, nbox) handle the oversampled boxes (factors of both ends, seeds,
// traces); in the workgroups after them each of the first npart waves
// solves the particular problem of one subdomain (one-ended factorisation
// of Omega_i), in its own part_ld doubles of LDS.  The two sets share nothing, so their waves run side
// by side instead of one launch after the other.
__global__ void __launch_bounds__(128) k_local_w(Geo g, const Box* __restrict__ obox,
                                                 const Box* __restrict__ pbox, int nbox,
                                                 const Seed* __restrict__ seeds,
                                                 const double* __restrict__ logK,
                                                 double* __restrict__ K,
                                                 const double* __restrict__ f,
                                                 const double* __restrict__ bcv, double beta,
                                                 double* __restrict__ fac,
                                                 double* __restrict__ tcoup,
                                                 double* __restrict__ facp,
                                                 double* __restrict__ tcp,
                                                 double* __restrict__ Pk,
                                                 double* __restrict__ tr_u,
                                                 double* __restrict__ tr_phi,
                                                 double* __restrict__ tr_beta,
                                                 double* __restrict__ pbar,
                                                 double* __restrict__ ubar,
                                                 double* __restrict__ pibar,
                                                 double* __restrict__ fact, int npart,
                                                 int part_ld, int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ WaveSmem sm[2];
  const int L = lane_id(), wv = threadIdx.x >> 6;
  if (L == 0) sm[wv].flag = 0;
  const int b = blockIdx.x;
  if (b < nbox) {
    const Box B = obox[b];
    basis_box(g, B, seeds, logK, beta, fac, fact, tcoup, Pk, tr_u, tr_phi, tr_beta, dsm, sm);
  } else {
    // npart (1 or 2) subdomains per workgroup, one per wave, each in its own
    // part_ld doubles of LDS
    const int pi = npart * (b - nbox) + wv;
    if (wv < npart && pi < nbox) {
      const Box B = pbox[pi];
      particular_box(g, B, logK, K, f, bcv, beta, facp, tcp, pbar, ubar, pibar,
                     dsm + (size_t)wv * part_ld, sm[wv]);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && (sm[0].flag | sm[1].flag)) atomicOr(flags, sm[0].flag | sm[1].flag);
}

// Algorithm 1, Step 6: the oversampled boxes factored again with the
// smoothing Robin parameter (when it differs from the basis one), two waves
// per box as in k_local_w, into their own forward / backward inverses.
__global__ void __launch_bounds__(128) k_factor_w(Geo g, const Box* __restrict__ obox,
                                                  const double* __restrict__ logK, double beta,
                                                  double* __restrict__ fac,
                                                  double* __restrict__ fact, int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ WaveSmem sm[2];
  const int L = lane_id(), wv = threadIdx.x >> 6;
  if (L == 0) sm[wv].flag = 0;
  const Box B = obox[blockIdx.x];
  basis_box<true>(g, B, nullptr, logK, beta, fac, fact, nullptr, nullptr, nullptr, nullptr,
                  nullptr, dsm, sm);
  __syncthreads();
  if (threadIdx.x == 0 && (sm[0].flag | sm[1].flag)) atomicOr(flags, sm[0].flag | sm[1].flag);
}

// Factor blocks a box's smoothing solve needs first (the first ring slots of
// both halves on waves 0 and 1, the meeting block on wave 0): constant data,
// loaded early so that their memory latency overlaps other work.
template <int NT>
__device__ __forceinline__ void smooth_preload(const Box& B, const double* Wf, const double* Wt,
                                               double w[RING][HB], double zm[HB]) {
  const int wv = threadIdx.x >> 6;
  if (NT > 64 && wv < 2) twist_preload(twist_half(B, wv == 0 ? Wf : Wt, B.nblk / 2, wv == 1), w);
  if (threadIdx.x < 64) wload_block(block_src(Wt, B.nb, B.nblk), B.nblk / 2, zm);
}

// Steps 6-7 for one box: stage the box's data, build the right-hand side,
// solve with the two-ended block sweep (its halves on the first two waves
// when NT >= 128) and write p on Omega_i and Omega_i's Gamma fluxes.
template <int NT>
__device__ __forceinline__ void smooth_box(const Geo& g, const Box& B, const double* __restrict__ K,
                                           const double* __restrict__ f,
                                           const double* __restrict__ bcv, double beta,
                                           const double* Wf, const double* Wt,
                                           const double* __restrict__ tcoup, double* p,
                                           double* gflux, double w[RING][HB], const double zm[HB],
                                           double* dsm) {
  SmoothLds r = carve_smooth(dsm, B, g.kc);
  stage_smooth<NT>(g, B, r, K, p, f, gflux, bcv, tcoup);
  bsync<NT>();
  smooth_rhs<NT>(g, B, r, beta, r.b.X);
  bsync<NT>();
  sweep_twisted<NT>(B, Wf, Wt, r.b, r.b.Z, w, zm);
  smooth_out<NT>(g, B, r, r.b.X, beta, p, gflux);
}

// Steps 6-7: one color phase of the smoothing sweep, one workgroup of NT
// threads (64, 128 or 256, chosen by the autotuner) per box.  The result
// does not depend on NT.
template <int NT>
__global__ void __launch_bounds__(NT) k_smooth_w(Geo g, const Box* __restrict__ boxes,
                                                 const double* __restrict__ K,
                                                 const double* __restrict__ f,
                                                 const double* __restrict__ bcv, double beta,
                                                 const double* __restrict__ fac,
                                                 const double* __restrict__ fact,
                                                 const double* __restrict__ tcoup,
                                                 double* __restrict__ p,
                                                 double* __restrict__ gflux) {
  extern __shared__ __align__(16) double dsm[];
  const Box B = boxes[blockIdx.x];
  double w[RING][HB], zm[HB];
  smooth_preload<NT>(B, fac + B.fac, fact + B.fac, w, zm);
  smooth_box<NT>(g, B, K, f, bcv, beta, fac + B.fac, fact + B.fac, tcoup, p, gflux, w, zm, dsm);
}

// All colour phases of nphase / ncol smoothing steps in one cooperative
// launch.  In phase k (colour k % ncol) workgroup b takes boxes b, b + G,
// b + 2G, ... of that colour (G workgroups, all resident at once), and a
// grid-wide barrier separates the phases, so that a phase reads the state
// its predecessors wrote.  After each box a workgroup already loads the
// first factor blocks of its next box, also across the barrier (factors do
// not change during smoothing).  Every workgroup passes every barrier.
template <int NT>
__global__ void __launch_bounds__(NT) k_smooth_grid(Geo g, const Box* __restrict__ boxes,
                                                    SmoothPhases ph, int nphase,
                                                    const double* __restrict__ K,
                                                    const double* __restrict__ f,
                                                    const double* __restrict__ bcv, double beta,
                                                    const double* __restrict__ fac,
                                                    const double* __restrict__ fact,
                                                    const double* __restrict__ tcoup, double* p,
                                                    double* gflux) {
  extern __shared__ __align__(16) double dsm[];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int G = gridDim.x, b0 = blockIdx.x;
  auto count = [&](int k) { return ph.off[k % ph.ncol + 1] - ph.off[k % ph.ncol]; };
  auto box_at = [&](int k, int j) { return ph.off[k % ph.ncol] + j; };
  auto preload = [&](int bi, double w[RING][HB], double zm[HB]) {
    const Box B = boxes[bi];
    smooth_preload<NT>(B, fac + B.fac, fact + B.fac, w, zm);
  };
  double w[RING][HB], zm[HB];
  int bi = b0 < count(0) ? box_at(0, b0) : -1;
  if (bi >= 0) preload(bi, w, zm);
  for (int k = 0; k < nphase; ++k) {
    const int n = count(k);
    const int n1 = k + 1 < nphase ? count(k + 1) : 0;
    for (int j = b0; j < n; j += G) {
      const Box B = boxes[bi];
      smooth_box<NT>(g, B, K, f, bcv, beta, fac + B.fac, fact + B.fac, tcoup, p, gflux, w, zm, dsm);
      bi = j + G < n ? box_at(k, j + G) : (b0 < n1 ? box_at(k + 1, b0) : -1);
      if (bi >= 0) preload(bi, w, zm);
    }
    if (b0 >= n && b0 < n1) {
      bi = box_at(k + 1, b0);
      preload(bi, w, zm);
    }
    grid.sync();
  }
}

template <typename KF>
hipError_t set_lds(KF kern, size_t bytes) {
  if (bytes > 64 * 1024)
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
  return hipSuccess;
}

}  // namespace

size_t wave_basis_lds_bytes(int m0, int m1, int nrhs, int kc) {
  return sizeof(double) * basis_lds_doubles(m0, m1, nrhs, kc);
}

size_t wave_lds_bytes(int m0, int m1, int nrhs, int kc) {
  return sizeof(double) * box_lds_doubles(m0, m1, nrhs, kc);
}

size_t wave_smooth_lds_bytes(int m0, int m1, int kc) { return sizeof(double) * smooth_lds_doubles(m0, m1, kc); }

hipError_t launch_local_w(const Geo& g, const Box* obox, const Box* pbox, int nbox,
                          const Seed* seeds, const double* logK, double* K, const double* f,
                          const double* bcv,
                          double beta, double* fac, double* tcoup, double* facp, double* tcp,
                          double* Pk, double* tr_u, double* tr_phi, double* tr_beta, double* pbar,
                          double* ubar, double* pibar, double* fact, int* flags, size_t lds,
                          size_t lds_part, hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  hipError_t e = set_lds(k_local_w, lds);
  if (e != hipSuccess) return e;
  if (!fact) return hipErrorInvalidValue;
  // Two subdomains per workgroup when the boxes outnumber the CUs several
  // times over (the launch is throughput-bound and a second wave per
  // workgroup costs no LDS); one when every box has a CU of its own and
  // the basis workgroups' latency decides.
  int dev = 0, ncu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int part_ld = (int)((lds_part / sizeof(double) + 1) / 2 * 2);  // 16-byte aligned waves
  const int npart = (nbox > 2 * ncu && (size_t)2 * part_ld * sizeof(double) <= lds) ? 2 : 1;
  if ((size_t)part_ld * sizeof(double) > lds) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_local_w, dim3(nbox + (nbox + npart - 1) / npart), dim3(128), lds, s, g, obox,
                     pbox, nbox, seeds, logK, K, f, bcv, beta, fac, tcoup, facp, tcp, Pk, tr_u,
                     tr_phi, tr_beta, pbar, ubar, pibar, fact, npart, part_ld, flags);
  return hipGetLastError();
}

hipError_t launch_factor_w(const Geo& g, const Box* obox, int nbox, const double* logK,
                           double beta, double* fac, double* fact, int* flags, size_t lds,
                           hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  if (!fac || !fact) return hipErrorInvalidValue;
  hipError_t e = set_lds(k_factor_w, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_factor_w, dim3(nbox), dim3(128), lds, s, g, obox, logK, beta, fac, fact,
                     flags);
  return hipGetLastError();
}

hipError_t launch_smooth_w(const Geo& g, const Box* boxes, int nmem,
                           const double* K, const double* f, const double* bcv, double beta,
                           const double* fac, const double* fact, const double* tcoup, double* scr,
                           double* p, double* gflux, size_t lds, int nt, hipStream_t s) {
  (void)scr;
  if (nmem <= 0) return hipSuccess;
  if (!fact) return hipErrorInvalidValue;
  hipError_t e;
#define MRCM_SMOOTH_NT(N)                                                                     \
  e = set_lds(k_smooth_w<N>, lds);                                                            \
  if (e != hipSuccess) return e;                                                              \
  hipLaunchKernelGGL(k_smooth_w<N>, dim3(nmem), dim3(N), lds, s, g, boxes, K, f, bcv,          \
                     beta, fac, fact, tcoup, p, gflux);
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

hipError_t launch_smooth_grid(const Geo& g, const Box* boxes, const SmoothPhases& ph, int nphase, const double* K, const double* f,
                              const double* bcv, double beta, const double* fac, const double* fact,
                              const double* tcoup, double* p, double* gflux, size_t lds, int nt,
                              int max_groups, hipStream_t s) {
  if (nphase <= 0) return hipSuccess;
  if (!fact || ph.ncol <= 0 || ph.ncol > 8 || max_groups < 0) return hipErrorInvalidValue;
  int nbox = 0;
  for (int c = 0; c < ph.ncol; ++c) nbox = std::max(nbox, ph.off[c + 1] - ph.off[c]);
  if (nbox <= 0) return hipSuccess;
  int dev = 0, ncu = 0, coop = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (!coop) return hipErrorNotSupported;
  Geo gg = g;
  SmoothPhases pp = ph;
  void* args[] = {&gg, &boxes, &pp, &nphase, &K, &f, &bcv, &beta, &fac, &fact, &tcoup, &p, &gflux};
  auto go = [&](auto kern, int N) -> hipError_t {
    hipError_t r = set_lds(kern, lds);
    if (r != hipSuccess) return r;
    int per_cu = 0;
    r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, N, lds);
    if (r != hipSuccess) return r;
    long long grid = std::min<long long>(nbox, (long long)per_cu * ncu);
    if (max_groups > 0) grid = std::min<long long>(grid, max_groups);
    if (grid <= 0) return hipErrorCooperativeLaunchTooLarge;
    return hipLaunchCooperativeKernel((const void*)kern, dim3((unsigned)grid), dim3(N), args, lds, s);
  };
  if (nt == 64) return go(k_smooth_grid<64>, 64);
  if (nt == 128) return go(k_smooth_grid<128>, 128);
  if (nt == 256) return go(k_smooth_grid<256>, 256);
  return hipErrorInvalidValue;
}

}  // namespace mrcm
