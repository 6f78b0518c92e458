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

#include <algorithm>

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

// One workgroup per (interface, equation row); each entry of the row (one
// column per seed of the two subdomains, then the right-hand side) is a sum
// over the interface faces, taken by a group of MG lanes: each lane adds
// the faces t = lane, lane + MG, ... and the group sums its lanes in a fixed
// order.  All loads of a round are in flight together.
constexpr int MG = 16;

__global__ void __launch_bounds__(256) k_moments(Geo g, const Iface* __restrict__ ifc,
                                                 const Seed* __restrict__ basis,
                                                 const int* __restrict__ seed_off,
                                                 const double* __restrict__ tr_u,
                                                 const double* __restrict__ tr_phi,
                                                 const double* __restrict__ tr_beta,
                                                 const double* __restrict__ ubar,
                                                 const double* __restrict__ pibar,
                                                 double* __restrict__ AB, int ldab, int kl, int ku,
                                                 double* __restrict__ rhs, BcrMap bm) {
  const Iface F = ifc[blockIdx.x];
  const int rr = blockIdx.y;
  const int nrow = 2 * F.nbasis;
  if (rr >= nrow) return;  // uniform over the workgroup
  const int qi = 2 * F.axis + 1, qj = 2 * F.axis;
  const int ni = seed_off[F.i + 1] - seed_off[F.i];
  const int nj = seed_off[F.j + 1] - seed_off[F.j];
  const int per_row = ni + nj + 1;  // entries + rhs
  int ilo[3], ihi[3];
  omega_box(g, F.i, ilo, ihi);
  int nf = 1;
  for (int b = 0; b < g.d; ++b)
    if (b != F.axis) nf *= g.S[b];
  const int kind = rr / F.nbasis;  // 0 flux, 1 pressure
  const Seed mu = basis[F.basis0 + rr % F.nbasis];
  const int row = F.row0 + rr;
  const int lg = threadIdx.x & (MG - 1), grp = threadIdx.x / MG, ngrp = blockDim.x / MG;
  for (int e0 = 0; e0 < per_row; e0 += ngrp) {
    const int e = e0 + grp;
    const bool valid = e < per_row;
    double acc = 0.0;
    int col = -1;
    if (valid && e < ni + nj) {
      const bool side_i = e < ni;
      const int sub = side_i ? F.i : F.j;
      const int k = side_i ? e : e - ni;
      const int q = side_i ? qi : qj;
      col = seed_off[sub] + k;
      const long long base = (long long)col * g.gstride + g.gside_off[q];
      const long long bbase = (long long)sub * g.gstride + g.gside_off[q];
      for (int t = lg; t < nf; t += MG) {
        int c[3];
        gface_cell(ilo, ihi, qi, t, c);
        const double w_t = g.area * seed_value(g, mu, ilo, ihi, c);
        const double v = kind == 0 ? tr_u[base + t] : tr_beta[bbase + t] * tr_u[base + t] + tr_phi[base + t];
        acc += w_t * v;
      }
      if (kind == 1 && !side_i) acc = -acc;
    } else if (valid) {
      const long long bi = (long long)F.i * g.gstride + g.gside_off[qi];
      const long long bj = (long long)F.j * g.gstride + g.gside_off[qj];
      for (int t = lg; t < nf; t += MG) {
        int c[3];
        gface_cell(ilo, ihi, qi, t, c);
        const double w_t = g.area * seed_value(g, mu, ilo, ihi, c);
        const double v = kind == 0 ? ubar[bi + t] + ubar[bj + t] : pibar[bi + t] - pibar[bj + t];
        acc += w_t * v;
      }
    }
#pragma unroll
    for (int off = MG / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (valid && lg == 0) {
      if (e < ni + nj) {
        if (g.neumann && row == 0) acc = (col == 0) ? 1.0 : 0.0;
        if (bm.dst) {
          const long long d = bm.dst[(long long)row * bm.dstw + e];
          if (d >= 0) bm.pool[d] = acc;
        } else if (bm.pool) {
          // straight into the reduction's layer blocks: D, L or U of the
          // equation's layer (block tridiagonal by construction)
          const int li = bm.row_lvl[row], lc = bm.col_lvl[col];
          const int kb = lc == li ? 0 : (lc == li - 1 ? 1 : 2);
          bm.pool[(long long)(kb * bm.M + li) * bm.bp * bm.bp + (long long)bm.row_loc[row] * bm.bp +
                  bm.col_loc[col]] = acc;
        } else {
          AB[(long long)row * (kl + ku + 1) + (col - row + kl)] = acc;
        }
      } else {
        const double v = (g.neumann && row == 0) ? 0.0 : -acc;
        if (bm.dst) bm.pool[bm.rdst[row]] = v;
        else if (bm.pool) bm.vec[(long long)bm.row_lvl[row] * bm.bp + bm.row_loc[row]] = v;
        else rhs[row] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Banded LU with partial pivoting (rows j..j+kl), one workgroup.
// Input RB: row i holds columns i-kl .. i+ku at RB[i*(kl+ku+1) + c-i+kl].
// Output UR: row i of U holds columns i .. i+kl+ku at UR[i*(kl+ku+1) + c-i];
// the right-hand side is eliminated alongside, then back substitution.

constexpr int LU_THREADS = 1024;

// x in [0, 2m) -> x mod m, without an integer division.
__device__ __forceinline__ int wrap(int x, int m) { return x >= m ? x - m : x; }

// Unblocked variant: the active (kl+1) x (kl+ku+1) window lives in LDS.
__global__ void __launch_bounds__(LU_THREADS) k_bandlu(const double* __restrict__ RB, int n,
                                                       int kl, int ku,
                                                       const double* __restrict__ rhs,
                                                       double* __restrict__ UR,
                                                       double* __restrict__ x, int* flags) {
  extern __shared__ double smem[];
  const int R = kl + 1;
  const int CW = kl + ku + 1;
  const int WI = kl + ku + 1;
  double* win = smem;              // R * CW, slot (i mod R, c mod CW)
  double* zr = win + R * CW;       // R
  double* lm = zr + R;             // R (multipliers)
  __shared__ int s_piv;
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  if (tid == 0) s_flag = 0;
  auto orig = [&](int i, int c) -> double {
    if (c < 0 || c >= n || i < 0 || i >= n) return 0.0;
    const int t = c - i + kl;
    if (t < 0 || t >= WI) return 0.0;
    return RB[(long long)i * WI + t];
  };
  for (int e = tid; e < R * CW; e += LU_THREADS) {
    const int i = e / CW, c = e - (e / CW) * CW;
    win[i * CW + c] = orig(i, c);
  }
  for (int i = tid; i < R; i += LU_THREADS) zr[i] = (i < n) ? rhs[i] : 0.0;
  __syncthreads();
  int jr = 0, jc = 0;  // slots of row j and column j
  for (int j = 0; j < n; ++j) {
    const int km = min(kl, n - 1 - j);
    if (tid < 64) {
      double best = -1.0;
      int bi = j;
      for (int t = tid; t <= km; t += 64) {
        const double v = fabs(win[wrap(jr + t, R) * CW + jc]);
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
    const int prs = wrap(jr + (pr - j), R);
    if (pr != j) {
      for (int c = tid; c < CW; c += LU_THREADS) {
        const int cs = wrap(jc + c, CW);
        const double a = win[jr * CW + cs];
        win[jr * CW + cs] = win[prs * CW + cs];
        win[prs * CW + cs] = a;
      }
      if (tid == 0) {
        const double a = zr[jr];
        zr[jr] = zr[prs];
        zr[prs] = a;
      }
    }
    __syncthreads();
    const double piv = win[jr * CW + jc];
    for (int i = 1 + tid; i <= km; i += LU_THREADS)
      lm[i] = (piv != 0.0) ? win[wrap(jr + i, R) * CW + jc] / piv : 0.0;
    __syncthreads();
    const int ncols = CW - 1;
    for (int e = tid; e < km * (ncols + 1); e += LU_THREADS) {
      const int ii = e / (ncols + 1), c = e - ii * (ncols + 1);
      const int i = 1 + ii;
      const int rs = wrap(jr + i, R);
      if (c < ncols) {
        const int cs = wrap(jc + 1 + c, CW);
        win[rs * CW + cs] -= lm[i] * win[jr * CW + cs];
      } else {
        zr[rs] -= lm[i] * zr[jr];
      }
    }
    for (int c = tid; c < CW; c += LU_THREADS)
      UR[(long long)j * CW + c] = (j + c < n) ? win[jr * CW + wrap(jc + c, CW)] : 0.0;
    __syncthreads();
    if (tid == 0) x[j] = zr[jr];
    // slide: row j's slot takes row j + kl + 1, column j's slot column j + CW
    const int nr = j + kl + 1;
    for (int c = tid; c < CW; c += LU_THREADS)
      win[jr * CW + wrap(jc + 1 + c, CW)] = (nr < n) ? orig(nr, j + 1 + c) : 0.0;
    if (tid == 0) zr[jr] = (nr < n) ? rhs[nr] : 0.0;
    for (int i = 1 + tid; i <= kl; i += LU_THREADS) win[wrap(jr + i, R) * CW + jc] = 0.0;
    __syncthreads();
    jr = wrap(jr + 1, R);
    jc = wrap(jc + 1, CW);
  }
  double* xs = smem;
  __syncthreads();
  if (tid < 64) {
    int js = (n - 1) % CW;
    for (int j = n - 1; j >= 0; --j) {
      double acc = 0.0;
      for (int c = 1 + tid; c < CW; c += 64)
        if (j + c < n) acc += UR[(long long)j * CW + c] * xs[wrap(js + c, CW)];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      const double v = (x[j] - acc) / UR[(long long)j * CW];
      if (tid == 0) {
        xs[js] = v;
        x[j] = v;
      }
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_wave_barrier();
      js = (js == 0) ? CW - 1 : js - 1;
    }
  }
  __syncthreads();
  if (tid == 0 && s_flag) atomicOr(flags, s_flag);
}

// Wave-wide maximum of a 64-bit key (all lanes receive it), using DPP
// quad permutations and row rotations within rows of 16 lanes, then the
// gfx950 permlane16/permlane32 swaps across rows.
__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

template <int CTRL>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v & 0xffffffffu), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

__device__ __forceinline__ unsigned long long wave_max_key(unsigned long long k) {
  k = umax64(k, dpp64<0xB1>(k));   // quad_perm(1,0,3,2)
  k = umax64(k, dpp64<0x4E>(k));   // quad_perm(2,3,0,1)
  k = umax64(k, dpp64<0x124>(k));  // row_ror:4
  k = umax64(k, dpp64<0x128>(k));  // row_ror:8
  {
    const int lo = (int)(unsigned)(k & 0xffffffffu), hi = (int)(unsigned)(k >> 32);
    const auto l2 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h2 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    k = umax64(((unsigned long long)(unsigned)h2[0] << 32) | (unsigned)l2[0],
               ((unsigned long long)(unsigned)h2[1] << 32) | (unsigned)l2[1]);
  }
  {
    const int lo = (int)(unsigned)(k & 0xffffffffu), hi = (int)(unsigned)(k >> 32);
    const auto l2 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h2 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    k = umax64(((unsigned long long)(unsigned)h2[0] << 32) | (unsigned)l2[0],
               ((unsigned long long)(unsigned)h2[1] << 32) | (unsigned)l2[1]);
  }
  return k;
}

// Pivot key: |v| (non-negative, so its bit pattern orders like the value)
// with the low 11 mantissa bits replaced by 2047 - row offset, so that the
// maximum picks the largest magnitude and, among equal truncated
// magnitudes, the smallest row.  Non-candidates use key 0.
__device__ __forceinline__ unsigned long long pivot_key(double v, int t) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(v));
  return (b & ~0x7FFull) | (unsigned long long)(2047 - t);
}

// Broadcast lane `src` (wave-uniform) of a double to all lanes.
__device__ __forceinline__ double bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

// Blocked variant: panels of BNB columns.  Window rows [j0, j0+H) and
// columns [j0, j0+WC) live in LDS in circular slots, H = BNB + kl,
// WC = BNB + kl + ku.  Per panel: wave 0 factors the H x BNB panel with
// partial pivoting in registers; every thread then applies the panel's row
// permutation (as one gather) and the unit-lower triangular solve to one
// column right of the panel (U12), then the register-tiled rank-BNB update
// of the trailing window, then the window slides by BNB rows / columns (the
// entering rows are prefetched into registers at the start of the panel).
constexpr int BNB = 16;
constexpr int BT = 512;
constexpr int PF = 8;   // prefetched values per thread

__global__ void __launch_bounds__(BT) k_bandlu_blocked(const double* __restrict__ RB, int n,
                                                       int kl, int ku,
                                                       const double* __restrict__ rhs,
                                                       double* __restrict__ UR,
                                                       double* __restrict__ x, int* flags) {
  extern __shared__ double smem[];
  const int H = BNB + kl;
  const int WC = BNB + kl + ku;
  const int LDW = WC + 1;
  const int WI = kl + ku + 1;
  const int WU = kl + ku + 1;
  double* win = smem;            // H * LDW
  double* zr = win + H * LDW;    // H
  double* swp = zr + H;          // 2 * BNB
  __shared__ int piv[BNB];       // pivot row offsets (relative to j0)
  __shared__ int perm_src[128];  // row permutation of the panel (offsets)
  __shared__ int mv_pos[2 * BNB], mv_src[2 * BNB];
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  if (tid == 0) s_flag = 0;
  auto orig = [&](int i, int c) -> double {
    if (c < 0 || c >= n || i < 0 || i >= n) return 0.0;
    const int t = c - i + kl;
    if (t < 0 || t >= WI) return 0.0;
    return RB[(long long)i * WI + t];
  };
  for (int e = tid; e < H * WC; e += BT) {
    const int i = e / WC, c = e - (e / WC) * WC;
    win[i * LDW + c] = orig(i, c);
  }
  for (int i = tid; i < H; i += BT) zr[i] = (i < n) ? rhs[i] : 0.0;
  __syncthreads();
  int j0h = 0, j0w = 0;  // slots of row j0 and column j0
  for (int j0 = 0; j0 < n; j0 += BNB) {
    const int nbp = min(BNB, n - j0);
    const int j1 = j0 + nbp;
    auto RS = [&](int t) { return wrap(j0h + t, H); };  // slot of row j0 + t, t < H
    auto CS = [&](int t) { int v = j0w + t; v = wrap(v, WC); return wrap(v, WC); };  // column j0 + t
    // prefetch the rows entering the window after this panel
    double pf[PF];
    const int npf = nbp * WC;
    const bool use_pf = npf <= PF * BT;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * BT;
      pf[q] = 0.0;
      if (use_pf && e < npf) {
        const int rr = e / WC;
        pf[q] = orig(j0 + H + rr, j1 + (e - rr * WC));
      }
    }
    // (A) panel factorisation by wave 0
    if (tid < 64) {
      const int t0 = lane, t1 = lane + 64;  // row offsets from j0
      const bool v0 = t0 < H && j0 + t0 < n;
      const bool v1 = t1 < H && j0 + t1 < n;
      const int s0 = v0 ? RS(t0) : 0, s1 = v1 ? RS(t1) : 0;
      double a0[BNB], a1[BNB];
#pragma unroll
      for (int c = 0; c < BNB; ++c) {
        const int cs = CS(c);
        a0[c] = (v0 && c < nbp) ? win[s0 * LDW + cs] : 0.0;
        a1[c] = (v1 && c < nbp) ? win[s1 * LDW + cs] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < BNB; ++k) {
        if (k >= nbp) break;
        const int lim = min(k + kl, n - 1 - j0);
        unsigned long long key = 0;
        if (v0 && t0 >= k && t0 <= lim) key = pivot_key(a0[k], t0);
        if (v1 && t1 >= k && t1 <= lim) key = umax64(key, pivot_key(a1[k], t1));
        key = wave_max_key(key);
        const int p = 2047 - (int)(key & 0x7FFull);
        if (lane == 0) piv[k] = p;
        // pivot row (lane p & 63, first or second slot) and row k (lane k,
        // first slot) broadcast with readlane; exchange them in registers
        const int pl = p & 63;
        const bool phi = p >= 64;
        double prow[BNB];
#pragma unroll
        for (int c = 0; c < BNB; ++c) prow[c] = bcast(phi ? a1[c] : a0[c], pl);
        if (p != k) {
          double krow[BNB];
#pragma unroll
          for (int c = 0; c < BNB; ++c) krow[c] = bcast(a0[c], k);
          const bool isk = t0 == k, isp0 = !phi && t0 == p, isp1 = phi && t1 == p;
#pragma unroll
          for (int c = 0; c < BNB; ++c) {
            a0[c] = isk ? prow[c] : (isp0 ? krow[c] : a0[c]);
            a1[c] = isp1 ? krow[c] : a1[c];
          }
        }
        const double pk = prow[k];
        if (lane == 0 && !(pk != 0.0)) s_flag |= kFlagSingular;
        const double ip = (pk != 0.0) ? 1.0 / pk : 0.0;
        {
          const bool e0 = v0 && t0 > k, e1 = v1 && t1 > k;
          const double l0 = e0 ? a0[k] * ip : 0.0;
          const double l1 = e1 ? a1[k] * ip : 0.0;
          a0[k] = e0 ? l0 : a0[k];
          a1[k] = e1 ? l1 : a1[k];
#pragma unroll
          for (int c = 0; c < BNB; ++c)
            if (c > k) {
              a0[c] = fma(-l0, prow[c], a0[c]);
              a1[c] = fma(-l1, prow[c], a1[c]);
            }
        }
      }
#pragma unroll
      for (int c = 0; c < BNB; ++c) {
        if (c < nbp) {
          const int cs = CS(c);
          if (v0) win[s0 * LDW + cs] = a0[c];
          if (v1) win[s1 * LDW + cs] = a1[c];
        }
      }
      // net row permutation of the panel: position t takes row perm_src[t]
      if (t0 < H) perm_src[t0] = t0;
      if (t1 < H) perm_src[t1] = t1;
      wave_lds_sync();
      if (lane == 0) {
        for (int k = 0; k < nbp; ++k) {
          const int p = piv[k];
          const int tmp = perm_src[k];
          perm_src[k] = perm_src[p];
          perm_src[p] = tmp;
        }
      }
      wave_lds_sync();
      if (lane < 2 * BNB) {
        const int pos = (lane < BNB) ? lane : piv[lane - BNB];
        const bool ok = (lane < BNB) ? lane < nbp : (lane - BNB) < nbp;
        mv_pos[lane] = ok ? pos : -1;
        mv_src[lane] = ok ? perm_src[pos] : -1;
      }
    }
    __syncthreads();
    // (B)+(C) permutation and unit-lower solve on each column right of the panel (+ rhs)
    const int ncr = WC - nbp;  // columns j1 .. j0+WC-1
    for (int cc = tid; cc <= ncr; cc += BT) {
      double* col;
      int stride;
      if (cc < ncr) {
        col = win + CS(nbp + cc);
        stride = LDW;
      } else {
        col = zr;
        stride = 1;
      }
      double mv[2 * BNB];
#pragma unroll
      for (int q = 0; q < 2 * BNB; ++q) {
        const int src = __builtin_amdgcn_readfirstlane(mv_src[q]);
        mv[q] = col[RS(max(src, 0)) * stride];
      }
#pragma unroll
      for (int q = 0; q < 2 * BNB; ++q) {
        const int src = __builtin_amdgcn_readfirstlane(mv_src[q]);
        const int pos = __builtin_amdgcn_readfirstlane(mv_pos[q]);
        if (src >= 0 && src != pos) col[RS(pos) * stride] = mv[q];
      }
      double u[BNB];
#pragma unroll
      for (int k = 0; k < BNB; ++k) u[k] = col[RS(min(k, nbp - 1)) * stride];
#pragma unroll
      for (int k = 0; k < BNB; ++k) {
        const int ck = CS(k);
#pragma unroll
        for (int i = k + 1; i < BNB; ++i) u[i] -= win[RS(min(i, nbp - 1)) * LDW + ck] * u[k];
      }
#pragma unroll
      for (int k = 0; k < BNB; ++k)
        if (k < nbp) col[RS(k) * stride] = u[k];
    }
    __syncthreads();
    // (D) trailing update, rows [j1, j0+H), columns [j1, j0+WC) and the rhs
    // column.  Work items are (strip of 8 rows, column); consecutive threads
    // take consecutive columns, so the U12 reads and the updates hit distinct
    // LDS banks and the L21 reads are broadcasts.
    {
      const int nr = H - nbp;
      const int nc = ncr + 1;  // + rhs
      const int ns = (nr + 7) / 8;
      for (int t = tid; t < ns * nc; t += BT) {
        const int st = t / nc;
        const int cc = t - st * nc;
        const int ib = st * 8;
        const bool isr = (cc == ncr);
        const double* ubase = isr ? zr : win + CS(nbp + cc);
        const int ustr = isr ? 1 : LDW;
        int rs[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) rs[a] = RS(nbp + min(ib + a, nr - 1));
        double acc[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) acc[a] = 0.0;
        for (int k = 0; k < nbp; ++k) {
          const int ck = CS(k), rk = RS(k);
          const double uv = ubase[rk * ustr];
#pragma unroll
          for (int a = 0; a < 8; ++a) acc[a] = fma(win[rs[a] * LDW + ck], uv, acc[a]);
        }
        double* obase = isr ? zr : win + CS(nbp + cc);
#pragma unroll
        for (int a = 0; a < 8; ++a)
          if (ib + a < nr) obase[rs[a] * ustr] -= acc[a];
      }
    }
    __syncthreads();
    // (E) U rows and eliminated rhs out
    for (int e = tid; e < nbp * WU; e += BT) {
      const int r = e / WU, t = e - r * WU;
      UR[(long long)(j0 + r) * WU + t] = (j0 + r + t < n) ? win[RS(r) * LDW + CS(r + t)] : 0.0;
    }
    for (int r = tid; r < nbp; r += BT) x[j0 + r] = zr[RS(r)];
    __syncthreads();
    // (F) slide: retired rows' slots get rows +H, retired columns' slots get columns +WC
    for (int e = tid; e < (H - nbp) * nbp; e += BT) {
      const int i = e / nbp, c = e - i * nbp;
      win[RS(nbp + i) * LDW + CS(WC + c)] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * BT;
      if (use_pf && e < npf) {
        const int rr = e / WC;
        win[RS(rr) * LDW + CS(nbp + e - rr * WC)] = pf[q];
      }
    }
    if (!use_pf)
      for (int e = tid; e < npf; e += BT) {
        const int rr = e / WC;
        win[RS(rr) * LDW + CS(nbp + e - rr * WC)] = orig(j0 + H + rr, j1 + e - rr * WC);
      }
    for (int r = tid; r < nbp; r += BT) zr[RS(r)] = (j0 + H + r < n) ? rhs[j0 + H + r] : 0.0;
    __syncthreads();
    j0h = RS(nbp);
    j0w = CS(nbp);
  }
  // back substitution, BNB rows at a time.  The U rows of the block are
  // staged in LDS (the next block's rows are prefetched into registers
  // meanwhile); partial sums with the known solutions by all threads, then
  // the triangular BNB x BNB part by wave 0, column by column: lane r keeps
  // its running right-hand side and x_c is broadcast with readlane.
  double* xs = smem;            // ring: x_c at slot c mod XR
  const int XR = WU + BNB;
  double* part = xs + XR;       // BNB partial sums
  double* ub = part + BNB;      // BNB x WU staged U rows
  const int last = ((n - 1) / BNB) * BNB;
  const int nub = BNB * WU;
  const bool pf_ok = nub <= PF * BT;
  double pu[PF];
  auto fetch = [&](int i0) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * BT;
      pu[q] = 0.0;
      if (e < nub) {
        const int r = i0 + e / WU;
        if (r < n) pu[q] = UR[(long long)i0 * WU + e];
      }
    }
  };
  if (pf_ok) fetch(last);
  __syncthreads();
  for (int i0 = last; i0 >= 0; i0 -= BNB) {
    const int nbr = min(BNB, n - i0);
    if (pf_ok) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int e = tid + q * BT;
        if (e < nub) ub[e] = pu[q];
      }
      if (i0 - BNB >= 0) fetch(i0 - BNB);
    } else {
      for (int e = tid; e < nub; e += BT) {
        const int r = i0 + e / WU;
        ub[e] = (r < n) ? UR[(long long)i0 * WU + e] : 0.0;
      }
    }
    __syncthreads();
    const int i0s = i0 % XR;
    {
      const int rr = tid >> 4, sub = tid & 15;
      double acc = 0.0;
      if (rr < nbr) {
        const int r = i0 + rr;
        for (int t = (nbr - rr) + sub; t < WU; t += 16) {
          const int sl = wrap(i0s + rr + t, XR);
          if (r + t < n) acc += ub[rr * WU + t] * xs[sl];
        }
      }
      for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
      if (sub == 0 && rr < nbr) part[rr] = x[i0 + rr] - acc;
    }
    __syncthreads();
    if (tid < 64) {
      double rsd = (lane < nbr) ? part[lane] : 0.0;
      double xv = 0.0;
      for (int c = nbr - 1; c >= 0; --c) {
        const double xc_local = (lane == c) ? rsd / ub[c * WU] : 0.0;
        const double xc = bcast(xc_local, c);
        if (lane == c) xv = xc;
        if (lane < c) rsd -= ub[lane * WU + (c - lane)] * xc;
      }
      if (lane < nbr) {
        xs[wrap(i0s + lane, XR)] = xv;
        x[i0 + lane] = xv;
      }
    }
    __syncthreads();
  }
  if (tid == 0 && s_flag) atomicOr(flags, s_flag);
}

// MRCM-O assembly: p = pbar + sum_k X_k P_k on each Omega_i and Gamma fluxes
// u = ubar + sum_k X_k u_k (equations eq:addu, eq:addp, eq:uhatphat), one
// launch: workgroups [0, nbp) the cells, the rest the Gamma faces.
__global__ void k_combine(Geo g, const int* __restrict__ seed_off, const double* __restrict__ X,
                          const double* __restrict__ Pk, const double* __restrict__ pbar,
                          double* __restrict__ p, const double* __restrict__ tr_u,
                          const double* __restrict__ ubar, double* __restrict__ gflux, int nbp) {
  if ((int)blockIdx.x < nbp) {
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
  } else {
    const long long e = (long long)(blockIdx.x - nbp) * blockDim.x + threadIdx.x;
    if (e >= (long long)g.nsub * g.gstride) return;
    const int sub = (int)(e / g.gstride), t = (int)(e % g.gstride);
    double v = ubar[e];
    for (int k = seed_off[sub]; k < seed_off[sub + 1]; ++k) v += X[k] * tr_u[(long long)k * g.gstride + t];
    gflux[e] = v;
  }
}

}  // namespace

hipError_t launch_moments(const Geo& g, const Iface* ifc, int nifc, int nrow_max, const Seed* basis,
                          const int* seed_off, const double* tr_u, const double* tr_phi,
                          const double* tr_beta, const double* ubar, const double* pibar,
                          double* AB, int ldab, int kl, int ku, double* rhs, hipStream_t s,
                          const BcrMap* bm) {
  if (nifc <= 0 || nrow_max <= 0) return hipSuccess;
  const BcrMap m = bm ? *bm : BcrMap{};
  hipLaunchKernelGGL(k_moments, dim3(nifc, nrow_max), dim3(256), 0, s, g, ifc, basis, seed_off, tr_u,
                     tr_phi, tr_beta, ubar, pibar, AB, ldab, kl, ku, rhs, m);
  return hipGetLastError();
}

hipError_t launch_bandlu_solve(double* RB, int ldab, int n, int kl, int ku, double* rhs, double* x,
                               int* ipiv, int* flags, hipStream_t s) {
  (void)ipiv;
  (void)ldab;
  if (n <= 0) return hipSuccess;
  double* UR = RB + (long long)n * (kl + ku + 1);  // U rows follow the input rows
  const size_t maxlds = 160 * 1024 - 256;
  const size_t lds_blk = sizeof(double) * ((size_t)(BNB + kl) * (BNB + kl + ku + 1) + (BNB + kl) + 2 * BNB);
  const size_t lds_bs = sizeof(double) * ((size_t)(kl + ku + 1) * (BNB + 1) + 2 * BNB);
  if (kl + BNB <= 128 && std::max(lds_blk, lds_bs) <= maxlds) {
    const size_t lds = std::max(lds_blk, lds_bs);
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)k_bandlu_blocked,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_bandlu_blocked, dim3(1), dim3(BT), lds, s, RB, n, kl, ku, rhs, UR, x, flags);
    return hipGetLastError();
  }
  const size_t lds = sizeof(double) * ((size_t)(kl + 1) * (kl + ku + 1) + 2 * (kl + 1));
  if (lds > maxlds) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_bandlu,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_bandlu, dim3(1), dim3(LU_THREADS), lds, s, RB, n, kl, ku, rhs, UR, x, flags);
  return hipGetLastError();
}

hipError_t launch_combine(const Geo& g, const int* seed_off, const double* X, const double* Pk,
                          const double* tr_u, const double* pbar, const double* ubar, double* p,
                          double* gflux, hipStream_t s) {
  const int ncell_o = g.S[0] * g.S[1] * (g.d == 3 ? g.S[2] : 1);
  const long long n1 = (long long)g.nsub * ncell_o;
  const long long n2 = (long long)g.nsub * g.gstride;
  const int nbp = (int)((n1 + 255) / 256), nbu = (int)((n2 + 255) / 256);
  if (nbp + nbu == 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)(nbp + nbu)), dim3(256), 0, s, g, seed_off, X, Pk, pbar,
                     p, tr_u, ubar, gflux, nbp);
  return hipGetLastError();
}

}  // namespace mrcm
