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
      AB[(long long)row * (kl + ku + 1) + (col - row + kl)] = acc;
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

// ---------------------------------------------------------------------------
// Banded LU with partial pivoting (rows j..j+kl), one workgroup.
// Input RB: row i holds columns i-kl .. i+ku at RB[i*(kl+ku+1) + c-i+kl].
// Output UR: row i of U holds columns i .. i+kl+ku at UR[i*(kl+ku+1) + c-i];
// the right-hand side is eliminated alongside, then back substitution.

constexpr int LU_THREADS = 1024;

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
    const int t = c - i + kl;
    if (t < 0 || t >= WI) return 0.0;
    return RB[(long long)i * WI + t];
  };
  for (int e = tid; e < R * CW; e += LU_THREADS) {
    const int i = e / CW, c = e % CW;
    W(i, c) = orig(i, c);
  }
  for (int i = tid; i < R; i += LU_THREADS) zr[i % R] = (i < n) ? rhs[i] : 0.0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int km = min(kl, n - 1 - j);
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
    const int ncols = CW - 1;
    for (int e = tid; e < km * (ncols + 1); e += LU_THREADS) {
      const int i = 1 + e / (ncols + 1), c = e % (ncols + 1);
      if (c < ncols) W(j + i, j + 1 + c) -= lm[i] * W(j, j + 1 + c);
      else zr[(j + i) % R] -= lm[i] * zr[j % R];
    }
    for (int c = tid; c < CW; c += LU_THREADS) UR[(long long)j * CW + c] = (j + c < n) ? W(j, j + c) : 0.0;
    __syncthreads();
    if (tid == 0) x[j] = zr[j % R];
    const int nr = j + kl + 1;
    for (int c = tid; c < CW; c += LU_THREADS) W(nr, j + 1 + c) = (nr < n) ? orig(nr, j + 1 + c) : 0.0;
    if (tid == 0) zr[nr % R] = (nr < n) ? rhs[nr] : 0.0;
    for (int i = 1 + tid; i <= kl; i += LU_THREADS) W(j + i, j + CW) = 0.0;
    __syncthreads();
  }
  double* xs = smem;
  __syncthreads();
  if (tid < 64) {
    for (int j = n - 1; j >= 0; --j) {
      double acc = 0.0;
      for (int c = 1 + tid; c < CW; c += 64)
        if (j + c < n) acc += UR[(long long)j * CW + c] * xs[(j + c) % CW];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      const double v = (x[j] - acc) / UR[(long long)j * CW];
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

// Blocked variant: panels of BNB columns.  Window rows [j0, j0+H) and
// columns [j0, j0+WC) live in LDS (circular slots), H = BNB + kl,
// WC = BNB + kl + ku.  Per panel: wave 0 factors the H x BNB panel with
// partial pivoting in registers; all threads apply the row interchanges and
// the unit-lower triangular solve to their columns (U12), then the
// register-tiled rank-BNB update of the trailing window, then the window
// slides by BNB rows / columns (next rows prefetched into registers).
constexpr int BNB = 16;
constexpr int BT = 256;
constexpr int PF = 16;  // prefetched values per thread

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
  __shared__ int piv[BNB];
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  if (tid == 0) s_flag = 0;
  auto WIN = [&](int i, int c) -> double& { return win[(i % H) * LDW + (c % WC)]; };
  auto orig = [&](int i, int c) -> double {
    if (c < 0 || c >= n || i < 0 || i >= n) return 0.0;
    const int t = c - i + kl;
    if (t < 0 || t >= WI) return 0.0;
    return RB[(long long)i * WI + t];
  };
  for (int e = tid; e < H * WC; e += BT) {
    const int i = e / WC, c = e % WC;
    WIN(i, c) = orig(i, c);
  }
  for (int i = tid; i < H; i += BT) zr[i % H] = (i < n) ? rhs[i] : 0.0;
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += BNB) {
    const int nbp = min(BNB, n - j0);
    const int j1 = j0 + nbp;  // next panel start
    // prefetch the rows entering the window after this panel
    double pf[PF];
    const int npf = nbp * WC;
    const bool use_pf = npf <= PF * BT;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * BT;
      pf[q] = 0.0;
      if (use_pf && e < npf) {
        const int r = j0 + H + e / WC;
        const int c = j1 + e % WC;
        pf[q] = orig(r, c);
      }
    }
    // (A) panel factorisation by wave 0
    if (tid < 64) {
      const int r0 = j0 + lane, r1 = j0 + lane + 64;
      const bool v0 = lane < H && r0 < n;
      const bool v1 = lane + 64 < H && r1 < n;
      double a0[BNB], a1[BNB];
#pragma unroll
      for (int c = 0; c < BNB; ++c) {
        a0[c] = (v0 && c < nbp) ? WIN(r0, j0 + c) : 0.0;
        a1[c] = (v1 && c < nbp) ? WIN(r1, j0 + c) : 0.0;
      }
#pragma unroll
      for (int k = 0; k < BNB; ++k) {
        if (k >= nbp) break;
        const int lim = min(j0 + k + kl, n - 1);
        double best = -1.0;
        int bi = 0x7fffffff;
        if (v0 && r0 >= j0 + k && r0 <= lim) { best = fabs(a0[k]); bi = r0; }
        if (v1 && r1 >= j0 + k && r1 <= lim) {
          const double t = fabs(a1[k]);
          if (t > best) { best = t; bi = r1; }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off);
          const int oi = __shfl_xor(bi, off);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const int p = bi;
        if (lane == 0) {
          piv[k] = p;
          if (!(best > 0.0)) s_flag |= kFlagSingular;
        }
        // exchange rows j0+k (lane k, first slot) and p through LDS
        const int rk = j0 + k;
        if (r0 == rk) {
#pragma unroll
          for (int c = 0; c < BNB; ++c) swp[c] = a0[c];
        }
        if (v0 && r0 == p) {
#pragma unroll
          for (int c = 0; c < BNB; ++c) swp[BNB + c] = a0[c];
        }
        if (v1 && r1 == p) {
#pragma unroll
          for (int c = 0; c < BNB; ++c) swp[BNB + c] = a1[c];
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        if (p != rk) {
          if (r0 == rk) {
#pragma unroll
            for (int c = 0; c < BNB; ++c) a0[c] = swp[BNB + c];
          }
          if (v0 && r0 == p) {
#pragma unroll
            for (int c = 0; c < BNB; ++c) a0[c] = swp[c];
          }
          if (v1 && r1 == p) {
#pragma unroll
            for (int c = 0; c < BNB; ++c) a1[c] = swp[c];
          }
        }
        const double pk = swp[BNB + k];
        const double ip = (pk != 0.0) ? 1.0 / pk : 0.0;
        if (v0 && r0 > rk) {
          const double l = a0[k] * ip;
          a0[k] = l;
#pragma unroll
          for (int c = 0; c < BNB; ++c)
            if (c > k) a0[c] -= l * swp[BNB + c];
        }
        if (v1 && r1 > rk) {
          const double l = a1[k] * ip;
          a1[k] = l;
#pragma unroll
          for (int c = 0; c < BNB; ++c)
            if (c > k) a1[c] -= l * swp[BNB + c];
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
      }
#pragma unroll
      for (int c = 0; c < BNB; ++c) {
        if (c < nbp) {
          if (v0) WIN(r0, j0 + c) = a0[c];
          if (v1) WIN(r1, j0 + c) = a1[c];
        }
      }
    }
    __syncthreads();
    // (B)+(C) interchanges and unit-lower solve on the columns right of the panel (+ rhs)
    const int ncr = WC - nbp;  // columns j1 .. j0+WC-1
    for (int cc = tid; cc <= ncr; cc += BT) {
      if (cc < ncr) {
        const int c = j1 + cc;
        for (int k = 0; k < nbp; ++k) {
          const int p = piv[k];
          if (p != j0 + k) {
            const double a = WIN(j0 + k, c);
            WIN(j0 + k, c) = WIN(p, c);
            WIN(p, c) = a;
          }
        }
        for (int k = 0; k < nbp; ++k) {
          const double a = WIN(j0 + k, c);
          for (int i = k + 1; i < nbp; ++i) WIN(j0 + i, c) -= WIN(j0 + i, j0 + k) * a;
        }
      } else {
        for (int k = 0; k < nbp; ++k) {
          const int p = piv[k];
          if (p != j0 + k) {
            const double a = zr[(j0 + k) % H];
            zr[(j0 + k) % H] = zr[p % H];
            zr[p % H] = a;
          }
        }
        for (int k = 0; k < nbp; ++k) {
          const double a = zr[(j0 + k) % H];
          for (int i = k + 1; i < nbp; ++i) zr[(j0 + i) % H] -= WIN(j0 + i, j0 + k) * a;
        }
      }
    }
    __syncthreads();
    // (D) trailing update, rows [j1, j0+H), columns [j1, j0+WC) and the rhs column
    {
      const int nr = H - nbp;
      const int nc = ncr + 1;  // + rhs
      const int tr = (nr + 3) / 4, tc = (nc + 3) / 4;
      for (int t = tid; t < tr * tc; t += BT) {
        const int ib = (t / tc) * 4, cb = (t % tc) * 4;
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        for (int k = 0; k < nbp; ++k) {
          double lv[4], uv[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) lv[a] = (ib + a < nr) ? WIN(j1 + ib + a, j0 + k) : 0.0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int cc = cb + b;
            uv[b] = (cc < ncr) ? WIN(j0 + k, j1 + cc) : (cc == ncr ? zr[(j0 + k) % H] : 0.0);
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = fma(lv[a], uv[b], acc[a][b]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          if (ib + a >= nr) continue;
          const int i = j1 + ib + a;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int cc = cb + b;
            if (cc < ncr) WIN(i, j1 + cc) -= acc[a][b];
            else if (cc == ncr) zr[i % H] -= acc[a][b];
          }
        }
      }
    }
    __syncthreads();
    // (E) U rows and eliminated rhs out
    for (int e = tid; e < nbp * WU; e += BT) {
      const int r = j0 + e / WU, t = e % WU;
      UR[(long long)r * WU + t] = (r + t < n) ? WIN(r, r + t) : 0.0;
    }
    for (int r = j0 + tid; r < j1; r += BT) x[r] = zr[r % H];
    __syncthreads();
    // (F) slide: retired rows' slots get rows +H, retired columns' slots get columns +WC
    for (int e = tid; e < (H - nbp) * nbp; e += BT) {
      const int i = j1 + e / nbp, c = j0 + WC + e % nbp;
      WIN(i, c) = 0.0;
    }
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * BT;
      if (use_pf && e < npf) WIN(j0 + H + e / WC, j1 + e % WC) = pf[q];
    }
    if (!use_pf)
      for (int e = tid; e < npf; e += BT) WIN(j0 + H + e / WC, j1 + e % WC) = orig(j0 + H + e / WC, j1 + e % WC);
    for (int r = j0 + H + tid; r < j0 + H + nbp; r += BT) zr[r % H] = (r < n) ? rhs[r] : 0.0;
    __syncthreads();
  }
  // back substitution, BNB rows at a time: partial sums by all threads,
  // then the triangular BNB x BNB part by wave 0
  double* xs = smem;            // ring of the last WU + BNB solutions
  const int XR = WU + BNB;
  double* part = smem + XR;     // BNB partial sums
  for (int i0 = ((n - 1) / BNB) * BNB; i0 >= 0; i0 -= BNB) {
    const int nbr = min(BNB, n - i0);
    // row r = i0 + tid / 16, 16 threads per row over columns >= i0 + nbr
    {
      const int rr = tid >> 4, sub = tid & 15;
      double acc = 0.0;
      if (rr < nbr) {
        const int r = i0 + rr;
        for (int t = (i0 + nbr - r) + sub; t < WU; t += 16)
          if (r + t < n) acc += UR[(long long)r * WU + t] * xs[(r + t) % XR];
      }
      for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
      if (sub == 0 && rr < nbr) part[rr] = x[i0 + rr] - acc;
    }
    __syncthreads();
    if (tid < 64) {
      for (int rr = nbr - 1; rr >= 0; --rr) {
        const int r = i0 + rr;
        double acc = 0.0;
        if (lane > rr && lane < nbr) acc = UR[(long long)r * WU + (lane - rr)] * xs[(i0 + lane) % XR];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        const double v = (part[rr] - acc) / UR[(long long)r * WU];
        if (lane == 0) {
          xs[r % XR] = v;
          x[r] = v;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
  }
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

hipError_t launch_bandlu_solve(double* RB, int ldab, int n, int kl, int ku, double* rhs, double* x,
                               int* ipiv, int* flags, hipStream_t s) {
  (void)ipiv;
  (void)ldab;
  if (n <= 0) return hipSuccess;
  double* UR = RB + (long long)n * (kl + ku + 1);  // U rows follow the input rows
  const size_t maxlds = 160 * 1024 - 256;
  const size_t lds_blk = sizeof(double) * ((size_t)(BNB + kl) * (BNB + kl + ku + 1) + (BNB + kl) + 2 * BNB);
  const size_t lds_bs = sizeof(double) * ((size_t)(kl + ku + 1) + 2 * BNB);
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
  hipLaunchKernelGGL(k_combine_p, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, g, seed_off,
                     X, Pk, pbar, p);
  const long long n2 = (long long)g.nsub * g.gstride;
  hipLaunchKernelGGL(k_combine_u, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, g, seed_off,
                     X, tr_u, ubar, gflux);
  return hipGetLastError();
}

}  // namespace mrcm
