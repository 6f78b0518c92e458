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
#include "local_common.h"

namespace mrcm {
namespace {

constexpr int NBW = 32;
constexpr int HB = 16;

struct WaveSmem {
  double row[2][NBW];
  double col[2][NBW];
  double z[kMaxRhs][NBW];
  double diag[NBW], tx[NBW], tprev[NBW], tnext[NBW];
  int flag;
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ void wsync() { __syncthreads(); }

__device__ __forceinline__ double half_swap(double v) { return __shfl_xor(v, 32); }

// Global coordinates of in-block cell a of block j (2-D: lines along x).
__device__ __forceinline__ void wblock_cell(const Box& B, int j, int a, int c[3]) {
  c[0] = B.lo[0] + a;
  c[1] = B.lo[1] + j;
  c[2] = 0;
}

__device__ __forceinline__ int wcell_loc(const Box& B, const int c[3]) {
  const int m0 = B.hi[0] - B.lo[0];
  return (c[0] - B.lo[0]) + m0 * (c[1] - B.lo[1]);
}

// Block coefficients of block j into LDS: diag, tx (to x+1), tnext (to y+1).
__device__ __forceinline__ void wload_coefs(const Geo& g, const Box& B, const double* K,
                                            double beta, int j, WaveSmem& sm) {
  const int L = lane_id();
  if (L < B.nb) {
    int c[3];
    wblock_cell(B, j, L, c);
    CellCoef cc = cell_coef(g, B, K, c, beta);
    sm.diag[L] = cc.diag;
    sm.tx[L] = cc.tp[0];
    sm.tnext[L] = cc.tp[1];
  } else if (L < NBW) {
    sm.diag[L] = 1.0;
    sm.tx[L] = 0.0;
    sm.tnext[L] = 0.0;
  }
}

// S_j (column c, my half) into w; w holds W_{j-1} on entry when j > 0.
__device__ __forceinline__ void wbuild(int nb, bool first, const WaveSmem& sm, double w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const double tc = sm.tprev[c];
#pragma unroll
  for (int i = 0; i < HB; ++i) {
    const int r = HB * h + i;
    double v;
    if (r >= nb || c >= nb) {
      v = (r == c) ? 1.0 : 0.0;
    } else {
      v = (r == c) ? sm.diag[c] : (r == c - 1) ? -sm.tx[r] : (r == c + 1) ? -sm.tx[c] : 0.0;
      if (!first) v -= sm.tprev[r] * tc * w[i];
    }
    w[i] = v;
  }
}

// In-place Gauss-Jordan inversion of the block held in w.  Each step
// publishes pivot row k (one element per lane of the owning half) and pivot
// column k (the 16 registers of the two lanes holding column k) to LDS.
__device__ __forceinline__ void wgj(int nb, WaveSmem& sm, double w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
#pragma unroll
  for (int k = 0; k < NBW; ++k) {
    if (k >= nb) break;
    double* rk = sm.row[k & 1];
    double* ck = sm.col[k & 1];
    if (h == (k >> 4)) rk[c] = w[k & 15];
    if (c == k) {
#pragma unroll
      for (int i = 0; i < HB; ++i) ck[HB * h + i] = w[i];
    }
    wsync();
    const double a = rk[c];
    const double piv = rk[k];
    if (!(piv > 0.0) && L == 0) sm.flag |= kFlagNotPD;
    const double ip = 1.0 / piv;
    const double f = -(a * ip);
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const double v = ck[HB * h + i];
      w[i] = (c == k) ? -v * ip : fma(f, v, w[i]);
    }
    if (h == (k >> 4)) w[k & 15] = (c == k) ? ip : a * ip;
  }
  wsync();
}

// y_k = W z_k for k < nrhs (z in sm.z), W symmetric held in w.  Result for
// row r returned in both half-lanes of column r.
__device__ __forceinline__ double wgemv_one(const double w[HB], const double* z) {
  const int L = lane_id();
  const int h = L >> 5;
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < HB; ++i) acc = fma(w[i], z[HB * h + i], acc);
  return acc + half_swap(acc);
}

__device__ __forceinline__ void wload_block(const double* Wj, int nb, double w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
#pragma unroll
  for (int i = 0; i < HB; ++i) {
    const int r = HB * h + i;
    w[i] = (r < nb && c < nb) ? Wj[r * nb + c] : 0.0;
  }
}

// Forward sweep fused with the factorisation.  Right-hand sides in S
// (S[k*ncell + cell]) are overwritten by w_j; inverses written to Wg and
// couplings t_j (to block j+1) to Tg.
__device__ void wfactor_forward(const Geo& g, const Box& B, const double* K, double beta,
                                double* Wg, double* Tg, double* S, int nrhs, WaveSmem& sm) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb;
  double w[HB];
#pragma unroll
  for (int i = 0; i < HB; ++i) w[i] = 0.0;
  for (int j = 0; j < B.nblk; ++j) {
    wsync();
    if (L < NBW) sm.tprev[L] = (j > 0) ? sm.tnext[L] : 0.0;
    wsync();
    wload_coefs(g, B, K, beta, j, sm);
    wsync();
    if (L < nb) Tg[j * nb + L] = sm.tnext[L];
    wbuild(nb, j == 0, sm, w);
    wgj(nb, sm, w);
    double* Wj = Wg + (long long)j * nb * nb;
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const int r = HB * h + i;
      if (r < nb && c < nb) Wj[r * nb + c] = w[i];
    }
    // forward step for every right-hand side
    for (int e = L; e < nrhs * NBW; e += 64) {
      const int k = e / NBW, r = e % NBW;
      double v = 0.0;
      if (r < nb) {
        v = S[(long long)k * B.ncell + j * nb + r];
        if (j > 0) v += sm.tprev[r] * S[(long long)k * B.ncell + (j - 1) * nb + r];
      }
      sm.z[k][r] = v;
    }
    wsync();
    for (int k = 0; k < nrhs; ++k) {
      const double y = wgemv_one(w, sm.z[k]);
      if (h == 0 && c < nb) S[(long long)k * B.ncell + j * nb + c] = y;
    }
  }
  wsync();
}

// Forward sweep with cached inverses.
__device__ void wforward(const Box& B, const double* Wg, const double* Tg, double* S, int nrhs,
                         WaveSmem& sm) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb;
  double w[HB], wn[HB];
  wload_block(Wg, nb, wn);
  for (int j = 0; j < B.nblk; ++j) {
#pragma unroll
    for (int i = 0; i < HB; ++i) w[i] = wn[i];
    if (j + 1 < B.nblk) wload_block(Wg + (long long)(j + 1) * nb * nb, nb, wn);
    wsync();
    for (int e = L; e < nrhs * NBW; e += 64) {
      const int k = e / NBW, r = e % NBW;
      double v = 0.0;
      if (r < nb) {
        v = S[(long long)k * B.ncell + j * nb + r];
        if (j > 0) v += Tg[(j - 1) * nb + r] * S[(long long)k * B.ncell + (j - 1) * nb + r];
      }
      sm.z[k][r] = v;
    }
    wsync();
    for (int k = 0; k < nrhs; ++k) {
      const double y = wgemv_one(w, sm.z[k]);
      if (h == 0 && c < nb) S[(long long)k * B.ncell + j * nb + c] = y;
    }
  }
  wsync();
}

// Backward sweep with cached inverses.
__device__ void wbackward(const Box& B, const double* Wg, const double* Tg, double* S, int nrhs,
                          WaveSmem& sm) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb;
  double w[HB], wn[HB];
  if (B.nblk >= 2) wload_block(Wg + (long long)(B.nblk - 2) * nb * nb, nb, wn);
  for (int j = B.nblk - 2; j >= 0; --j) {
#pragma unroll
    for (int i = 0; i < HB; ++i) w[i] = wn[i];
    if (j >= 1) wload_block(Wg + (long long)(j - 1) * nb * nb, nb, wn);
    wsync();
    for (int e = L; e < nrhs * NBW; e += 64) {
      const int k = e / NBW, r = e % NBW;
      sm.z[k][r] = (r < nb) ? Tg[j * nb + r] * S[(long long)k * B.ncell + (j + 1) * nb + r] : 0.0;
    }
    wsync();
    for (int k = 0; k < nrhs; ++k) {
      const double y = wgemv_one(w, sm.z[k]);
      if (h == 0 && c < nb) S[(long long)k * B.ncell + j * nb + c] += y;
    }
  }
  wsync();
}

__device__ __forceinline__ void womega(const Geo& g, int sub, int lo[3], int hi[3]) {
  const int ix = sub % g.M[0], iy = sub / g.M[0];
  lo[0] = ix * g.S[0];
  hi[0] = lo[0] + g.S[0];
  lo[1] = iy * g.S[1];
  hi[1] = lo[1] + g.S[1];
  lo[2] = 0;
  hi[2] = 1;
}

__device__ __forceinline__ bool win_box(const Box& B, const int c[3]) {
  return c[0] >= B.lo[0] && c[0] < B.hi[0] && c[1] >= B.lo[1] && c[1] < B.hi[1];
}

__device__ __forceinline__ int wneighbor(const Geo& g, int sub, int q) {
  const int a = q >> 1, s = q & 1;
  const int ia = (a == 0) ? sub % g.M[0] : sub / g.M[0];
  const int t = ia + (s ? 1 : -1);
  if (t < 0 || t >= g.M[a]) return -1;
  const int stride = (a == 0) ? 1 : g.M[0];
  return sub + (s ? stride : -stride);
}

// Inner cell of face t on Gamma side q of Omega = [lo, hi) (2-D).
__device__ __forceinline__ void wgface(const int lo[3], const int hi[3], int q, int t, int c[3]) {
  const int a = q >> 1, s = q & 1;
  c[2] = 0;
  if (a == 0) {
    c[0] = s ? hi[0] - 1 : lo[0];
    c[1] = lo[1] + t;
  } else {
    c[1] = s ? hi[1] - 1 : lo[1];
    c[0] = lo[0] + t;
  }
}

// ------------------------------------------------------------------ kernels

__global__ void __launch_bounds__(64) k_basis_w(Geo g, const Box* __restrict__ boxes,
                                                const Seed* __restrict__ seeds,
                                                const double* __restrict__ K, double beta,
                                                double* __restrict__ fac,
                                                double* __restrict__ tcoup,
                                                double* __restrict__ scr, double* __restrict__ Pk,
                                                double* __restrict__ tr_u,
                                                double* __restrict__ tr_phi,
                                                double* __restrict__ tr_beta, int* flags) {
  __shared__ WaveSmem sm;
  const Box B = boxes[blockIdx.x];
  const int L = lane_id();
  if (L == 0) sm.flag = 0;
  const int nrhs = B.nrhs;
  double* S = scr + B.scr;
  for (long long e = L; e < (long long)nrhs * B.ncell; e += 64) S[e] = 0.0;
  wsync();
  for (int k = 0; k < nrhs; ++k) {
    const Seed sd = seeds[B.seed0 + k];
    const int a = sd.side >> 1, s = sd.side & 1;
    const int nf = (a == 0) ? B.hi[1] - B.lo[1] : B.hi[0] - B.lo[0];
    for (int t = L; t < nf; t += 64) {
      int c[3], o[3];
      if (a == 0) { c[0] = s ? B.hi[0] - 1 : B.lo[0]; c[1] = B.lo[1] + t; }
      else { c[1] = s ? B.hi[1] - 1 : B.lo[1]; c[0] = B.lo[0] + t; }
      c[2] = 0;
      o[0] = c[0]; o[1] = c[1]; o[2] = 0;
      o[a] += s ? 1 : -1;
      const double kc = K[gcell(g, c)];
      const double bt = robin_beta(g, a, kc, K[gcell(g, o)], beta);
      S[(long long)k * B.ncell + wcell_loc(B, c)] =
          robin_T(g, kc, bt) * seed_value(g, sd, B.lo, B.hi, c);
    }
  }
  wsync();
  double* Wg = fac + B.fac;
  double* Tg = tcoup + B.scr;  // per-box couplings share the scratch offsets (ncell each)
  wfactor_forward(g, B, K, beta, Wg, Tg, S, nrhs, sm);
  wbackward(B, Wg, Tg, S, nrhs, sm);
  int olo[3], ohi[3];
  womega(g, B.sub, olo, ohi);
  const int ncell_o = g.S[0] * g.S[1];
  for (int e = L; e < nrhs * ncell_o; e += 64) {
    const int k = e / ncell_o, t = e % ncell_o;
    int c[3] = {olo[0] + t % g.S[0], olo[1] + t / g.S[0], 0};
    Pk[(long long)(B.seed0 + k) * ncell_o + t] = S[(long long)k * B.ncell + wcell_loc(B, c)];
  }
  for (int q = 0; q < 4; ++q) {
    const int nf = (q >> 1) == 0 ? g.S[1] : g.S[0];
    const bool has = wneighbor(g, B.sub, q) >= 0;
    const int a = q >> 1, s = q & 1;
    for (int e = L; e < nrhs * nf; e += 64) {
      const int k = e / nf, t = e % nf;
      const long long oidx = (long long)(B.seed0 + k) * g.gstride + g.gside_off[q] + t;
      if (!has) {
        tr_u[oidx] = 0.0;
        tr_phi[oidx] = 0.0;
        continue;
      }
      int c[3], o[3];
      wgface(olo, ohi, q, t, c);
      o[0] = c[0]; o[1] = c[1]; o[2] = 0;
      o[a] += s ? 1 : -1;
      const double kc = K[gcell(g, c)], ko = K[gcell(g, o)];
      const double Pc = S[(long long)k * B.ncell + wcell_loc(B, c)];
      const double bt = robin_beta(g, a, kc, ko, beta);
      double u;
      if (win_box(B, o)) {
        u = g.area * kharm(kc, ko) / g.h * (Pc - S[(long long)k * B.ncell + wcell_loc(B, o)]) / g.area;
      } else {
        const Seed sd = seeds[B.seed0 + k];
        const double lam = (sd.side == q) ? seed_value(g, sd, B.lo, B.hi, c) : 0.0;
        u = robin_T(g, kc, bt) * (Pc - lam) / g.area;
      }
      const double pi = Pc - u * g.h / (2.0 * kc);
      tr_u[oidx] = u;
      tr_phi[oidx] = -bt * u + pi;
      if (k == 0) tr_beta[(long long)B.sub * g.gstride + g.gside_off[q] + t] = bt;
    }
  }
  wsync();
  if (L == 0 && sm.flag) atomicOr(flags, sm.flag);
}

__device__ void wphysical_rhs(const Geo& g, const Box& B, const double* K, const double* f,
                              const double* bcv, double* S) {
  for (int loc = lane_id(); loc < B.ncell; loc += 64) {
    const int m0 = B.hi[0] - B.lo[0];
    int c[3] = {B.lo[0] + loc % m0, B.lo[1] + loc / m0, 0};
    const int ci = gcell(g, c);
    double b = f[ci] * g.vol;
    for (int a = 0; a < 2; ++a)
      for (int s = 0; s < 2; ++s) {
        const int t = c[a] + (s ? 1 : -1);
        if (t >= 0 && t < g.n[a]) continue;
        const int side = 2 * a + s;
        const double val = bcv[g.bc_off[side] + bface_index(g, c, a)];
        if (g.bc_type[side]) b += 2.0 * K[ci] * g.area / g.h * val;
        else b -= g.area * val;
      }
    S[loc] = b;
  }
}

__global__ void __launch_bounds__(64) k_particular_w(Geo g, const Box* __restrict__ boxes,
                                                     const double* __restrict__ K,
                                                     const double* __restrict__ f,
                                                     const double* __restrict__ bcv, double beta,
                                                     double* __restrict__ fac,
                                                     double* __restrict__ tcoup,
                                                     double* __restrict__ scr,
                                                     double* __restrict__ pbar,
                                                     double* __restrict__ ubar,
                                                     double* __restrict__ pibar, int* flags) {
  __shared__ WaveSmem sm;
  const Box B = boxes[blockIdx.x];
  const int L = lane_id();
  if (L == 0) sm.flag = 0;
  double* S = scr + B.scr;
  wphysical_rhs(g, B, K, f, bcv, S);
  wsync();
  double* Wg = fac + B.fac;
  double* Tg = tcoup + B.scr;
  wfactor_forward(g, B, K, beta, Wg, Tg, S, 1, sm);
  wbackward(B, Wg, Tg, S, 1, sm);
  for (int t = L; t < B.ncell; t += 64) pbar[(long long)B.sub * B.ncell + t] = S[t];
  for (int q = 0; q < 4; ++q) {
    const int nf = (q >> 1) == 0 ? g.S[1] : g.S[0];
    const bool has = wneighbor(g, B.sub, q) >= 0;
    const int a = q >> 1, s = q & 1;
    for (int t = L; t < nf; t += 64) {
      const long long oidx = (long long)B.sub * g.gstride + g.gside_off[q] + t;
      if (!has) {
        ubar[oidx] = 0.0;
        pibar[oidx] = 0.0;
        continue;
      }
      int c[3], o[3];
      wgface(B.lo, B.hi, q, t, c);
      o[0] = c[0]; o[1] = c[1]; o[2] = 0;
      o[a] += s ? 1 : -1;
      const double kc = K[gcell(g, c)];
      const double bt = robin_beta(g, a, kc, K[gcell(g, o)], beta);
      const double u = robin_T(g, kc, bt) * S[wcell_loc(B, c)] / g.area;
      ubar[oidx] = u;
      pibar[oidx] = bt * u;
    }
  }
  wsync();
  if (L == 0 && sm.flag) atomicOr(flags, sm.flag);
}

// lambda = -beta u.n + pi on a Robin face of box B from the current state.
__device__ __forceinline__ double wlambda(const Geo& g, const Box& B, const double* K,
                                          const double* p, const double* gflux, double beta,
                                          const int c[3], int a, int s) {
  int o[3] = {c[0], c[1], 0};
  o[a] += s ? 1 : -1;
  const int ci = gcell(g, c), oi = gcell(g, o);
  const double kc = K[ci], ko = K[oi];
  const double bt = robin_beta(g, a, kc, ko, beta);
  if (g.l > 0) {
    const double u = g.area * kharm(kc, ko) / g.h * (p[ci] - p[oi]) / g.area;
    const double pi = p[ci] - u * g.h / (2.0 * kc);
    return -bt * u + pi;
  }
  const int q = 2 * a + s;
  const int j = wneighbor(g, B.sub, q);
  int jlo[3], jhi[3];
  womega(g, j, jlo, jhi);
  const int t = (a == 0) ? o[1] - jlo[1] : o[0] - jlo[0];
  const double uj = gflux[(long long)j * g.gstride + g.gside_off[q ^ 1] + t];
  const double pij = p[oi] - uj * g.h / (2.0 * ko);
  return bt * uj + pij;
}

__global__ void __launch_bounds__(64) k_smooth_w(Geo g, const Box* __restrict__ boxes,
                                                 const int* __restrict__ members,
                                                 const double* __restrict__ K,
                                                 const double* __restrict__ f,
                                                 const double* __restrict__ bcv, double beta,
                                                 const double* __restrict__ fac,
                                                 const double* __restrict__ tcoup,
                                                 double* __restrict__ scr, double* __restrict__ p,
                                                 double* __restrict__ gflux) {
  __shared__ WaveSmem sm;
  const Box B = boxes[members[blockIdx.x]];
  const int L = lane_id();
  double* S = scr + B.scr;
  const int m0 = B.hi[0] - B.lo[0];
  for (int loc = L; loc < B.ncell; loc += 64) {
    int c[3] = {B.lo[0] + loc % m0, B.lo[1] + loc / m0, 0};
    const int ci = gcell(g, c);
    const double kc = K[ci];
    double b = f[ci] * g.vol;
    for (int a = 0; a < 2; ++a)
      for (int s = 0; s < 2; ++s) {
        const int kind = face_kind(g, B, c, a, s);
        if (kind == kFaceInterior) continue;
        const int side = 2 * a + s;
        if (kind == kFaceRobin) {
          int o[3] = {c[0], c[1], 0};
          o[a] += s ? 1 : -1;
          const double bt = robin_beta(g, a, kc, K[gcell(g, o)], beta);
          b += robin_T(g, kc, bt) * wlambda(g, B, K, p, gflux, beta, c, a, s);
        } else {
          const double val = bcv[g.bc_off[side] + bface_index(g, c, a)];
          if (kind == kFaceDir) b += 2.0 * kc * g.area / g.h * val;
          else b -= g.area * val;
        }
      }
    S[loc] = b;
  }
  wsync();
  const double* Wg = fac + B.fac;
  const double* Tg = tcoup + B.scr;
  wforward(B, Wg, Tg, S, 1, sm);
  wbackward(B, Wg, Tg, S, 1, sm);
  int olo[3], ohi[3];
  womega(g, B.sub, olo, ohi);
  for (int q = 0; q < 4; ++q) {
    if (wneighbor(g, B.sub, q) < 0) continue;
    const int nf = (q >> 1) == 0 ? g.S[1] : g.S[0];
    const int a = q >> 1, s = q & 1;
    for (int t = L; t < nf; t += 64) {
      int c[3], o[3];
      wgface(olo, ohi, q, t, c);
      o[0] = c[0]; o[1] = c[1]; o[2] = 0;
      o[a] += s ? 1 : -1;
      const double kc = K[gcell(g, c)], ko = K[gcell(g, o)];
      const double xc = S[wcell_loc(B, c)];
      double u;
      if (win_box(B, o)) {
        u = g.area * kharm(kc, ko) / g.h * (xc - S[wcell_loc(B, o)]) / g.area;
      } else {
        const double lam = wlambda(g, B, K, p, gflux, beta, c, a, s);
        u = robin_T(g, kc, robin_beta(g, a, kc, ko, beta)) * (xc - lam) / g.area;
      }
      gflux[(long long)B.sub * g.gstride + g.gside_off[q] + t] = u;
    }
  }
  wsync();
  const int ncell_o = g.S[0] * g.S[1];
  for (int t = L; t < ncell_o; t += 64) {
    int c[3] = {olo[0] + t % g.S[0], olo[1] + t / g.S[0], 0};
    p[gcell(g, c)] = S[wcell_loc(B, c)];
  }
}

}  // namespace

hipError_t launch_basis_w(const Geo& g, const Box* boxes, int nbox, const Seed* seeds,
                          const double* K, double beta, double* fac, double* tcoup, double* scr,
                          double* Pk, double* tr_u, double* tr_phi, double* tr_beta, int* flags,
                          hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_basis_w, dim3(nbox), dim3(64), 0, s, g, boxes, seeds, K, beta, fac, tcoup,
                     scr, Pk, tr_u, tr_phi, tr_beta, flags);
  return hipGetLastError();
}

hipError_t launch_particular_w(const Geo& g, const Box* boxes, int nbox, const double* K,
                               const double* f, const double* bcv, double beta, double* fac,
                               double* tcoup, double* scr, double* pbar, double* ubar,
                               double* pibar, int* flags, hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_particular_w, dim3(nbox), dim3(64), 0, s, g, boxes, K, f, bcv, beta, fac,
                     tcoup, scr, pbar, ubar, pibar, flags);
  return hipGetLastError();
}

hipError_t launch_smooth_w(const Geo& g, const Box* boxes, const int* members, int nmem,
                           const double* K, const double* f, const double* bcv, double beta,
                           const double* fac, const double* tcoup, double* scr, double* p,
                           double* gflux, hipStream_t s) {
  if (nmem <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_smooth_w, dim3(nmem), dim3(64), 0, s, g, boxes, members, K, f, bcv, beta,
                     fac, tcoup, scr, p, gflux);
  return hipGetLastError();
}

}  // namespace mrcm
