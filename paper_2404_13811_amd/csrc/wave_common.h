// Shared pieces of the one-wavefront-per-box 2-D local kernels (FP64 and
// FP32-with-refinement forms): LDS layout of a box, coefficient loading,
// the Gauss-Jordan block inverse in the two-half-wave register layout, and
// geometry helpers.  See local_wave.hip for the algorithm.
#pragma once
#include "local_common.h"

namespace mrcm {
namespace wave {

constexpr int NBW = 32;
constexpr int HB = 16;
constexpr int RING = 4;

struct WaveSmem {
  double row[2][NBW];
  double col[2][NBW];
  int flag;
};

// Dynamic LDS carve-up of one box.
struct BoxLds {
  double* Kt;   // (m0 + 2) x (m1 + 2) permeabilities, one-cell halo
  double* Dg;   // ncell diagonal of A
  double* Tx;   // ncell coupling to the x+1 neighbour (0 at the box edge)
  double* Tn;   // ncell coupling to the next block (y+1)
  double* X;    // nrhs x ncell right-hand sides / solutions
  double* Z;    // nrhs x NBW staging of one block
  int m0, m1;
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Single-wave synchronisation through LDS: wait for this wave's LDS
// operations; the wave barrier keeps the compiler from moving memory
// operations across it.
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0) only
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double half_swap(double v) { return __shfl_xor(v, 32); }

__host__ __device__ inline size_t box_lds_doubles(int m0, int m1, int nrhs) {
  const int nc = m0 * m1;
  return (size_t)(m0 + 2) * (m1 + 2) + 3 * (size_t)nc + (size_t)nrhs * nc + (size_t)nrhs * NBW;
}

__device__ __forceinline__ BoxLds carve(double* base, const Box& B, int nrhs) {
  BoxLds s;
  s.m0 = B.hi[0] - B.lo[0];
  s.m1 = B.hi[1] - B.lo[1];
  const int nc = s.m0 * s.m1;
  s.Kt = base;
  s.Dg = s.Kt + (s.m0 + 2) * (s.m1 + 2);
  s.Tx = s.Dg + nc;
  s.Tn = s.Tx + nc;
  s.X = s.Tn + nc;
  s.Z = s.X + (size_t)nrhs * nc;
  return s;
}

// K at global cell (x, y), which must lie in the box or its halo.
__device__ __forceinline__ double kat(const BoxLds& s, const Box& B, int x, int y) {
  return s.Kt[(y - B.lo[1] + 1) * (s.m0 + 2) + (x - B.lo[0] + 1)];
}

// Load the K tile and the matrix coefficients of the box into LDS.
__device__ void load_box(const Geo& g, const Box& B, const double* K, double beta, BoxLds& s) {
  const int L = lane_id();
  const int W2 = s.m0 + 2, H2 = s.m1 + 2;
  for (int e = L; e < W2 * H2; e += 64) {
    const int x = B.lo[0] - 1 + e % W2, y = B.lo[1] - 1 + e / W2;
    s.Kt[e] = (x >= 0 && x < g.n[0] && y >= 0 && y < g.n[1]) ? K[x + g.n[0] * y] : 1.0;
  }
  wsync();
  const int nc = s.m0 * s.m1;
  for (int loc = L; loc < nc; loc += 64) {
    const int x = B.lo[0] + loc % s.m0, y = B.lo[1] + loc / s.m0;
    const double kc = kat(s, B, x, y);
    double diag = 0.0, tx = 0.0, tn = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int sd = 0; sd < 2; ++sd) {
        const int ox = x + (a == 0 ? (sd ? 1 : -1) : 0);
        const int oy = y + (a == 1 ? (sd ? 1 : -1) : 0);
        const int t = a == 0 ? ox : oy;
        if (t < 0 || t >= g.n[a]) {
          if (g.bc_type[2 * a + sd]) diag += 2.0 * kc * g.area / g.h;
          continue;
        }
        const double ko = kat(s, B, ox, oy);
        const bool inside = ox >= B.lo[0] && ox < B.hi[0] && oy >= B.lo[1] && oy < B.hi[1];
        if (inside) {
          const double T = g.area * kharm(kc, ko) / g.h;
          diag += T;
          if (sd) {
            if (a == 0) tx = T;
            else tn = T;
          }
        } else {
          diag += robin_T(g, kc, robin_beta(g, a, kc, ko, beta));
        }
      }
    s.Dg[loc] = diag;
    s.Tx[loc] = tx;
    s.Tn[loc] = tn;
  }
  wsync();
}

// S_j (column c, my half) into w; w holds W_{j-1} on entry when j > 0.
__device__ __forceinline__ void wbuild(int nb, int j, const BoxLds& s, double w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const double* D = s.Dg + j * nb;
  const double* Tx = s.Tx + j * nb;
  const double* Tp = s.Tn + (j - 1) * nb;
  const double tc = (j > 0 && c < nb) ? Tp[c] : 0.0;
#pragma unroll
  for (int i = 0; i < HB; ++i) {
    const int r = HB * h + i;
    double v;
    if (r >= nb || c >= nb) {
      v = (r == c) ? 1.0 : 0.0;
    } else {
      v = (r == c) ? D[c] : (r == c - 1) ? -Tx[r] : (r == c + 1) ? -Tx[c] : 0.0;
      if (j > 0) v -= Tp[r] * tc * w[i];
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

__device__ __forceinline__ void womega(const Geo& g, int sub, int lo[3], int hi[3]) {
  const int ix = sub % g.M[0], iy = sub / g.M[0];
  lo[0] = ix * g.S[0];
  hi[0] = lo[0] + g.S[0];
  lo[1] = iy * g.S[1];
  hi[1] = lo[1] + g.S[1];
  lo[2] = 0;
  hi[2] = 1;
}

__device__ __forceinline__ bool win_box(const Box& B, int x, int y) {
  return x >= B.lo[0] && x < B.hi[0] && y >= B.lo[1] && y < B.hi[1];
}

__device__ __forceinline__ int wneighbor(const Geo& g, int sub, int q) {
  const int a = q >> 1, sd = q & 1;
  const int ia = (a == 0) ? sub % g.M[0] : sub / g.M[0];
  const int t = ia + (sd ? 1 : -1);
  if (t < 0 || t >= g.M[a]) return -1;
  const int stride = (a == 0) ? 1 : g.M[0];
  return sub + (sd ? stride : -stride);
}

// Inner cell of face t on side q of [lo, hi) (2-D).
__device__ __forceinline__ void wgface(const int lo[3], const int hi[3], int q, int t, int& x, int& y) {
  const int a = q >> 1, sd = q & 1;
  if (a == 0) {
    x = sd ? hi[0] - 1 : lo[0];
    y = lo[1] + t;
  } else {
    y = sd ? hi[1] - 1 : lo[1];
    x = lo[0] + t;
  }
}

__device__ __forceinline__ int bloc(const Box& B, const BoxLds& s, int x, int y) {
  return (x - B.lo[0]) + s.m0 * (y - B.lo[1]);
}

// Physical right-hand side (source, boundary data) of box B into out.
__device__ void physical_rhs(const Geo& g, const Box& B, const BoxLds& s, const double* f,
                             const double* bcv, double* out) {
  const int nc = s.m0 * s.m1;
  for (int loc = lane_id(); loc < nc; loc += 64) {
    const int x = B.lo[0] + loc % s.m0, y = B.lo[1] + loc / s.m0;
    const int ci = x + g.n[0] * y;
    double b = f[ci] * g.vol;
    const int c[3] = {x, y, 0};
    for (int a = 0; a < 2; ++a)
      for (int sd = 0; sd < 2; ++sd) {
        const int t = c[a] + (sd ? 1 : -1);
        if (t >= 0 && t < g.n[a]) continue;
        const int side = 2 * a + sd;
        const double val = bcv[g.bc_off[side] + bface_index(g, c, a)];
        if (g.bc_type[side]) b += 2.0 * kat(s, B, x, y) * g.area / g.h * val;
        else b -= g.area * val;
      }
    out[loc] = b;
  }
}

// lambda = -beta u.n + pi on the Robin face of box B at inside cell (x, y),
// normal along a, side sd, from the current global state (Section 3).
__device__ __forceinline__ double wlambda(const Geo& g, const Box& B, const BoxLds& s,
                                          const double* p, const double* gflux, double beta,
                                          int x, int y, int a, int sd) {
  const int ox = x + (a == 0 ? (sd ? 1 : -1) : 0), oy = y + (a == 1 ? (sd ? 1 : -1) : 0);
  const int ci = x + g.n[0] * y, oi = ox + g.n[0] * oy;
  const double kc = kat(s, B, x, y), ko = kat(s, B, ox, oy);
  const double bt = robin_beta(g, a, kc, ko, beta);
  if (g.l > 0) {
    const double u = g.area * kharm(kc, ko) / g.h * (p[ci] - p[oi]) / g.area;
    const double pi = p[ci] - u * g.h / (2.0 * kc);
    return -bt * u + pi;
  }
  const int q = 2 * a + sd;
  const int j = wneighbor(g, B.sub, q);
  int jlo[3], jhi[3];
  womega(g, j, jlo, jhi);
  const int t = (a == 0) ? oy - jlo[1] : ox - jlo[0];
  const double uj = gflux[(long long)j * g.gstride + g.gside_off[q ^ 1] + t];
  const double pij = p[oi] - uj * g.h / (2.0 * ko);
  return bt * uj + pij;
}


}  // namespace wave
}  // namespace mrcm
