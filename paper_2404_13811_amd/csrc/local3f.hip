// Kernels for 3-D local problems in the FP32 form: the plane-block factor
// of the diagonally scaled box matrix A^ = D^-1/2 A D^-1/2 is formed and
// applied in FP32, and every local solve is refined in FP64 on the
// unscaled two-point-flux matrix A:
//     x = 0;  repeat  r = b - A x (FP64);  x += D^-1/2 solve32(D^-1/2 r)
// until the componentwise backward error max_c |r_c| / (|A| |x| + |b|)_c
// is at most tol.  Steps 1-2 (seed solves, traces on Gamma_i, basis
// functions on Omega_i), Step 4 (particular problems), Step 6 (factor only)
// and one colour phase of the smoothing sweep (Steps 6-7).
//
// Layout as the FP64 kernels (local3.hip): one workgroup of NW wavefronts
// per box, lane c of wave v holding rows 16v .. 16v + 15 of column c of the
// padded 64 x 64 plane block, here in FP32; the block LDL^T recurrence
// S_j = D_j - t_{j-1} W_{j-1} t_{j-1} with W_j = S_j^{-1} formed in place by
// four-pivot Gauss-Jordan elimination with look-ahead.  The sweeps run on
// row blocks of the inverses (local3_common.h: one quad-reduced dot
// product per lane, one barrier per plane step).  What the FP32 form adds:
// the basis kernel converts each new inverse to row blocks within its wave
// and holds the first JC = 8 planes' (16 registers each per lane, 128 in
// all), so the back substitution and every refinement sweep read no factor
// from memory; a smoothing box holds 8, 4 or 0 planes' inverses (the
// autotuner's choice) across its refinement sweeps and reads the others in
// every sweep.  Inverses not held are read from the stored ones (nb x nb,
// row-major FP32).
#include "local3_common.h"
#include "pivot4.h"

namespace mrcm {
namespace {

constexpr int JC = 8;   // plane inverses held in registers (most)
constexpr int JCB = 2;  // those the basis kernel holds (three boxes per CU)

// Pivot data of one elimination step (two alternating buffers), as Gj3 of
// the FP64 kernels in FP32; vb and rs (1024 floats) also hold the per-wave
// partial sums of the block-vector products.  red: the waves' maxima of
// the backward error.
struct __align__(16) Gj3f {
  float vb[2][G3 * P3];
  float rs[2][P3 * G3];
  float pb[2][G3 * G3];
  double red[4];
  int flag;
};

__device__ __forceinline__ float* partials3f(Gj3f& sm) { return &sm.vb[0][0]; }

// LDS of one box in the FP32 form: the FP64 box (K tile, diagonal, plane
// couplings; s.X holds the FP64 solutions x, nrhs x ncell), then
struct Box3F {
  Box3 s;
  double* sd;   // ncell: D^-1/2
  double* Bv;   // ncell right-hand side (particular and smoothing boxes)
  float* Xf;    // nrhs x ncell: scaled residuals, then the FP32 corrections
  float* Tzf;   // ncell: scaled couplings to the next plane
  float* Zf;    // 2 x nrhs x 64: staged inputs of a sweep step (16-byte aligned)
};

__host__ __device__ inline size_t box3f_bytes(int m0, int m1, int m2, int nrhs, int nbv, int kc) {
  const size_t nc = (size_t)m0 * m1 * m2;
  const size_t d = kx3_doubles(kc, m0, m1, m2) + (size_t)(m0 + 2) * (m1 + 2) * (m2 + 2) + 2 * nc +
                   (size_t)nrhs * nc + nc + (size_t)nbv * nc;
  const size_t f = (size_t)nrhs * nc + nc + 2 * (size_t)(nrhs < 1 ? 1 : nrhs) * P3 + 4;
  return d * sizeof(double) + f * sizeof(float) + 16;
}

template <bool TS>
__device__ __forceinline__ Box3F carve3f(double* base, const Box& B, int nrhs, int nbv, int kc) {
  Box3F F;
  F.s = carve3<TS>(base, B, nrhs, kc);  // F.s.Z (FP64 staging) is not used
  const int nc = F.s.nc;
  F.sd = F.s.X + (size_t)nrhs * nc;
  F.Bv = F.sd + nc;
  F.Xf = reinterpret_cast<float*>(F.Bv + (size_t)nbv * nc);
  F.Tzf = F.Xf + (size_t)nrhs * nc;
  const uintptr_t z = reinterpret_cast<uintptr_t>(F.Tzf + nc);
  F.Zf = reinterpret_cast<float*>((z + 15) & ~uintptr_t(15));
  return F;
}

// D^-1/2 and the scaled plane couplings (after load_box3).
template <int NW>
__device__ __forceinline__ void scale3f(const Box3F& F) {
  constexpr int NT = 64 * NW;
  const Box3& s = F.s;
  const int nc = s.nc, nb = s.m0 * s.m1;
  for (int e = threadIdx.x; e < nc; e += NT) F.sd[e] = rcp3(sqrt(s.Dg[e]));
  bsync<NW>();
  for (int e = threadIdx.x; e < nc; e += NT)
    F.Tzf[e] = e + nb < nc ? (float)(s.Tz[e] * F.sd[e] * F.sd[e + nb]) : 0.0f;
  bsync<NW>();
}

// Scaled S_j = D^_j - t^_{j-1} W_{j-1} t^_{j-1} (the lane's 16 entries of
// column c), w holding W_{j-1} on entry when j > 0; identity outside the
// nb x nb block.  The couplings are scaled in FP64 and rounded once.
__device__ __forceinline__ void build3f(const Geo& g, const Box& B, const Box3F& F, int j, float w[R3]) {
  const Box3& s = F.s;
  const int c = lane3();
  const int r0 = R3 * wave3();
  const int nb = s.m0 * s.m1, m0 = s.m0;
  const bool cin = c < nb;
  const int cc = cin ? c : 0;
  const int xl = cc % m0;
  const double* sdj = F.sd + j * nb;
  const double sc = sdj[cc];
  const float dc = (float)(s.Dg[j * nb + cc] * sc * sc);
  const float txm = (cin && xl > 0) ? (float)(tplane(g, B, s, j, cc - 1, 0) * sc * sdj[cc - 1]) : 0.0f;
  const float txp = (cin && xl + 1 < m0) ? (float)(tplane(g, B, s, j, cc, 0) * sc * sdj[cc + 1]) : 0.0f;
  const float tym = (cin && cc >= m0) ? (float)(tplane(g, B, s, j, cc - m0, 1) * sc * sdj[cc - m0]) : 0.0f;
  const float typ = (cin && cc + m0 < nb) ? (float)(tplane(g, B, s, j, cc, 1) * sc * sdj[cc + m0]) : 0.0f;
  const float* tp = F.Tzf + (j > 0 ? j - 1 : 0) * nb;
  const float tcp = (j > 0 && cin) ? tp[cc] : 0.0f;
#pragma unroll
  for (int ii = 0; ii < R3; ++ii) {
    const int i = r0 + ii;
    float v = (i == c) ? dc : 0.0f;
    v -= (i == c - 1) ? txm : 0.0f;
    v -= (i == c + 1) ? txp : 0.0f;
    v -= (i == c - m0) ? tym : 0.0f;
    v -= (i == c + m0) ? typ : 0.0f;
    if (j > 0 && i < nb) v = fmaf(-tp[i] * tcp, w[ii], v);
    w[ii] = (i < nb && cin) ? v : (i == c ? 1.0f : 0.0f);
  }
}

// Four-pivot Gauss-Jordan inverse with look-ahead in FP32: the steps of
// gj3_pivot / gj3_rows / gj3_step of the FP64 kernels, on floats.
template <int NW, int K>
__device__ __forceinline__ void gj3f_pivot(Gj3f& sm, float w[R3], bool& bad) {
  constexpr int RI = K % R3;
  const int c = lane3_here();
  const int ck = c - K;
  const bool pc = ck >= 0 && ck < G3;
  float* vb = sm.vb[(K / G3) & 1];
  float* rs = sm.rs[(K / G3) & 1];
  float* pb = sm.pb[(K / G3) & 1];
  if (pc) *reinterpret_cast<float4*>(pb + ck * G3) = make_float4(w[RI], w[RI + 1], w[RI + 2], w[RI + 3]);
  const float sg = c < K ? -1.0f : 1.0f;
  *reinterpret_cast<float4*>(rs + c * G3) =
      make_float4(sg * w[RI], sg * w[RI + 1], sg * w[RI + 2], sg * w[RI + 3]);
  bsync<1>();  // the pivot block is read back by this wave only
  float P[G3][G3], r[G3], v[G3];
#pragma unroll
  for (int j = 0; j < G3; ++j)
#pragma unroll
    for (int m = 0; m < G3; ++m) P[m][j] = pb[j * G3 + m];
#pragma unroll
  for (int m = 0; m < G3; ++m) {
    const float wm = w[RI + m];
    const float unit = ck == m ? 1.0f : 0.0f;
    r[m] = pc ? unit : wm;
  }
  const PivBlock<float> q = piv_block(P);
  bad |= !(q.d0 > 0.0f && q.da > 0.0f && q.s0 > 0.0f && q.ds > 0.0f);
  piv_apply(q, r, v);
#pragma unroll
  for (int m = 0; m < G3; ++m) vb[m * P3 + c] = v[m];
}

template <int R0, int R1>
__device__ __forceinline__ void gj3f_rows(const float* rw, unsigned keep, const float v[G3], float w[R3]) {
#pragma unroll
  for (int ii = R0; ii < R1; ++ii) {
    const float4 cr = *reinterpret_cast<const float4*>(rw + ii * G3);
    float acc = __uint_as_float(__float_as_uint(w[ii]) & keep);
    acc = fmaf(-cr.x, v[0], acc);
    acc = fmaf(-cr.y, v[1], acc);
    acc = fmaf(-cr.z, v[2], acc);
    acc = fmaf(-cr.w, v[3], acc);
    w[ii] = acc;
  }
}

template <int NW, int K>
__device__ __forceinline__ void gj3f_step(int nb, Gj3f& sm, float w[R3], bool& bad) {
  constexpr int OWN = K / R3, RI = K % R3;
  constexpr int KN = K + G3, OWNN = KN / R3, RIN = KN % R3;
  const int c = lane3_here();
  const int wv = wave3();
  const float* vb = sm.vb[(K / G3) & 1];
  const float* rw = sm.rs[(K / G3) & 1] + R3 * wv * G3;
  const int ck = c - K;
  const bool pc = ck >= 0 && ck < G3;
  const unsigned keep = pc ? 0u : ~0u;
  float v[G3];
#pragma unroll
  for (int m = 0; m < G3; ++m) v[m] = vb[m * P3 + c];
  if constexpr (KN < R3 * NW) {
    gj3f_rows<RIN, RIN + G3>(rw, keep, v, w);
    if (KN < nb && wv == OWNN) gj3f_pivot<NW, KN>(sm, w, bad);
    gj3f_rows<0, RIN>(rw, keep, v, w);
    gj3f_rows<RIN + G3, R3>(rw, keep, v, w);
  } else {
    gj3f_rows<0, R3>(rw, keep, v, w);
  }
  if (wv == OWN) {
#pragma unroll
    for (int m = 0; m < G3; ++m) w[RI + m] = v[m];
  }
  bsync<NW>();
}

template <int NW, int K>
__device__ __forceinline__ void gj3f_steps(int nb, Gj3f& sm, float w[R3], bool& bad) {
  if constexpr (K < R3 * NW) {
    if (K < nb) {
      gj3f_step<NW, K>(nb, sm, w, bad);
      gj3f_steps<NW, K + G3>(nb, sm, w, bad);
    }
  }
}

template <int NW>
__device__ __forceinline__ void gj3f(int nb, Gj3f& sm, float w[R3]) {
  bool bad = false;
  if (wave3() == 0) gj3f_pivot<NW, 0>(sm, w, bad);
  bsync<NW>();
  gj3f_steps<NW, 0>(nb, sm, w, bad);
  if (bad && lane3() == 0) atomicOr(&sm.flag, kFlagNotPD);
  bsync<NW>();
}

// Row blocks from the elimination layout (lane c: W[16v + ii][c]); both
// layouts give wave v the rows 16v .. 16v + 15, so the exchange stays in
// the wave: four rounds through a 16 x 16 staging tile T of the wave's own.
__device__ __forceinline__ void gj_to_rb(const float w[R3], float wr[R3], float* T) {
  const int c = lane3();
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    if ((c >> 4) == qq) {
#pragma unroll
      for (int ii = 0; ii < R3; ++ii) T[ii * R3 + (c & 15)] = w[ii];
    }
    bsync<1>();
    if ((c & 3) == qq) {
#pragma unroll
      for (int ii = 0; ii < R3; ii += 4) {
        const float4 v = *reinterpret_cast<const float4*>(T + (c >> 2) * R3 + ii);
        wr[ii] = v.x;
        wr[ii + 1] = v.y;
        wr[ii + 2] = v.z;
        wr[ii + 3] = v.w;
      }
    }
    bsync<1>();
  }
}

// The row-block sweep vectors of a box in the FP32 form: the scaled work
// vectors Xf, the scaled plane couplings Tzf and the staged inputs Zf.
__device__ __forceinline__ RbSweep<float> rbv(const Box3F& F, int nrhs) {
  return RbSweep<float>{F.Xf, F.Tzf, F.Zf, F.s.nc, F.s.m2, nrhs};
}

__device__ __forceinline__ void store3f(float* Wj, int nb, const float w[R3]) {
  const int c = lane3(), r0 = R3 * wave3();
#pragma unroll
  for (int ii = 0; ii < R3; ++ii) {
    const int i = r0 + ii;
    if (i < nb && c < nb) Wj[i * nb + c] = w[ii];
  }
}

// Register cache of the plane inverses (row blocks).  Slots are addressed
// with compile-time indices only: the sweeps run their first JC planes as
// an unrolled loop, and a plane formed at a runtime index is written into
// its slot by selects (a conditional store per slot would be merged into a
// store through a selected address, which keeps the cache in scratch
// memory).
template <int JCN>
__device__ __forceinline__ void cclear(float wc[JC][R3]) {
#pragma unroll
  for (int jj = 0; jj < JCN; ++jj)
#pragma unroll
    for (int ii = 0; ii < R3; ++ii) wc[jj][ii] = 0.0f;
}

template <int JCN>
__device__ __forceinline__ void cput(float wc[JC][R3], int j, const float w[R3]) {
#pragma unroll
  for (int jj = 0; jj < JCN; ++jj)
#pragma unroll
    for (int ii = 0; ii < R3; ++ii) wc[jj][ii] = jj == j ? w[ii] : wc[jj][ii];
}

// Factor of the box fused with the forward sweep of the nrhs scaled
// right-hand sides in Xf (plane 0's input staged); inverses to Wg and, as
// row blocks, those of the first JCN planes to the register cache.
template <int NW, int JCN>
__device__ __forceinline__ void factor3f(const Geo& g, const Box& B, const Box3F& F, float* Wg, int nrhs,
                                         Gj3f& sm, float wc[JC][R3]) {
  const int nb = F.s.m0 * F.s.m1;
  float* T = partials3f(sm) + R3 * R3 * wave3();
  float w[R3];
#pragma unroll
  for (int i = 0; i < R3; ++i) w[i] = 0.0f;
  cclear<JCN>(wc);
  for (int j = 0; j < F.s.m2; ++j) {
    build3f(g, B, F, j, w);
    gj3f<NW>(nb, sm, w);
    store3f(Wg + (long long)j * nb * nb, nb, w);
    if (nrhs > 0) {
      // the pivot buffers are free until the next plane's elimination,
      // which starts after the forward step's barrier
      float wr[R3];
      gj_to_rb(w, wr, T);
      cput<JCN>(wc, j, wr);
      fwd_rb<NW>(rbv(F, nrhs), nb, j, wr);
    }
  }
}

// JCN: planes taken from the register cache (JC, or 0: every plane read
// from the stored inverses).
template <int NW, int JCN = JC>
__device__ __forceinline__ void backward3f(const Box3F& F, const float wc[JC][R3], const float* Wg, int nrhs) {
  const int nb = F.s.m0 * F.s.m1, m2 = F.s.m2;
  float wr[R3];
  for (int j = m2 - 2; j >= JCN; --j) {
    load_rb(Wg + (long long)j * nb * nb, nb, wr);
    bwd_rb<NW>(rbv(F, nrhs), nb, j, wr);
  }
#pragma unroll
  for (int j = JCN - 1; j >= 0; --j)
    if (j <= m2 - 2) bwd_rb<NW>(rbv(F, nrhs), nb, j, wc[j]);
}

// Forward sweep with the cached inverses (LOAD: the cache filled from the
// stored inverses on the way); plane 0's input staged.
// Filling the cache, loads run one plane ahead of the plane being applied
// (into the next slot).
template <int NW, bool LOAD, int JCN = JC>
__device__ __forceinline__ void forward3f(const Box3F& F, float wc[JC][R3], const float* Wg, int nrhs) {
  const int nb = F.s.m0 * F.s.m1, m2 = F.s.m2;
  if (LOAD && JCN > 0 && m2 > 0) load_rb(Wg, nb, wc[0]);
#pragma unroll
  for (int j = 0; j < JCN; ++j)
    if (j < m2) {
      if (LOAD && j + 1 < JCN && j + 1 < m2) load_rb(Wg + (long long)(j + 1) * nb * nb, nb, wc[j + 1]);
      fwd_rb<NW>(rbv(F, nrhs), nb, j, wc[j]);
    }
  float wr[R3];
  for (int j = JCN; j < m2; ++j) {
    load_rb(Wg + (long long)j * nb * nb, nb, wr);
    fwd_rb<NW>(rbv(F, nrhs), nb, j, wr);
  }
}

// Xf <- A^^-1 Xf with the cached inverses.
template <int NW, int JCN = JC>
__device__ __forceinline__ void solve3f(const Box3F& F, float wc[JC][R3], const float* Wg, int nrhs) {
  stage0_rb<NW>(rbv(F, nrhs), F.s.m0 * F.s.m1);
  forward3f<NW, false, JCN>(F, wc, Wg, nrhs);
  backward3f<NW, JCN>(F, wc, Wg, nrhs);
}

// x += D^-1/2 (FP32 correction), for the nrhs solutions.
template <int NW>
__device__ __forceinline__ void update3f(const Box3F& F, int nrhs) {
  const int nc = F.s.nc;
  for (int e = threadIdx.x; e < nrhs * nc; e += 64 * NW) F.s.X[e] += F.sd[e % nc] * (double)F.Xf[e];
  bsync<NW>();
}

__device__ __forceinline__ double wave_max3(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// r = b - A x in FP64 for the nrhs solutions in s.X (b: the seeds' right-
// hand sides when seeds is given, else Bv), D^-1/2 r into Xf, and the
// componentwise backward error over the box (the same value on every lane).
// A residual or iterate that is not finite gives an infinite error.
template <int NW>
__device__ __forceinline__ double resid3f(const Geo& g, const Box& B, const Box3F& F,
                                          const Seed* __restrict__ seeds, double beta, int nrhs,
                                          Gj3f& sm) {
  constexpr int NT = 64 * NW;
  const Box3& s = F.s;
  const int nc = s.nc, m0 = s.m0, m1 = s.m1, m2 = s.m2, nb = m0 * m1;
  double om = 0.0;
  // the couplings of a cell once, for all its right-hand sides
  for (int loc = threadIdx.x; loc < nc; loc += NT) {
    const int xl = loc % m0, yl = (loc / m0) % m1, j = loc / nb, a = loc - j * nb;
    const double dg = s.Dg[loc], sdl = F.sd[loc];
    const double txm = xl > 0 ? tplane(g, B, s, j, a - 1, 0) : 0.0;
    const double txp = xl + 1 < m0 ? tplane(g, B, s, j, a, 0) : 0.0;
    const double tym = yl > 0 ? tplane(g, B, s, j, a - m0, 1) : 0.0;
    const double typ = yl + 1 < m1 ? tplane(g, B, s, j, a, 1) : 0.0;
    const double tzm = j > 0 ? s.Tz[loc - nb] : 0.0;
    const double tzp = j + 1 < m2 ? s.Tz[loc] : 0.0;
    const int c[3] = {B.lo[0] + xl, B.lo[1] + yl, B.lo[2] + j};
    for (int k = 0; k < nrhs; ++k) {
      const double* x = s.X + (size_t)k * nc;
      double bv;
      if (seeds) {
        const Seed sd = seeds[B.seed0 + k];
        const int sa = sd.side >> 1;
        const bool on = pick3(c, sa) == ((sd.side & 1) ? pick3(B.hi, sa) - 1 : pick3(B.lo, sa));
        bv = on ? seed_face_b3(g, B, s, sd, beta, c) : 0.0;
      } else {
        bv = F.Bv[loc];
      }
      double ax = dg * x[loc], aa = fabs(ax), t;
      if (xl > 0) { t = txm * x[loc - 1]; ax -= t; aa += fabs(t); }
      if (xl + 1 < m0) { t = txp * x[loc + 1]; ax -= t; aa += fabs(t); }
      if (yl > 0) { t = tym * x[loc - m0]; ax -= t; aa += fabs(t); }
      if (yl + 1 < m1) { t = typ * x[loc + m0]; ax -= t; aa += fabs(t); }
      if (j > 0) { t = tzm * x[loc - nb]; ax -= t; aa += fabs(t); }
      if (j + 1 < m2) { t = tzp * x[loc + nb]; ax -= t; aa += fabs(t); }
      const double r = bv - ax;
      const double den = aa + fabs(bv);
      if (!(r - r == 0.0 && den - den == 0.0)) om = INFINITY;
      else if (den > 0.0) om = fmax(om, fabs(r) / den);
      F.Xf[k * nc + loc] = (float)(sdl * r);
    }
  }
  om = wave_max3(om);
  if (lane3() == 0) sm.red[wave3()] = om;
  bsync<NW>();
  double omega = sm.red[0];
#pragma unroll
  for (int u = 1; u < NW; ++u) omega = fmax(omega, sm.red[u]);
  return omega;
}

// Refinement after the first FP32 solve (x = D^-1/2 z already in s.X);
// returns the number of FP32 solves, the final backward error in omega.
template <int NW, int JCN = JC>
__device__ __forceinline__ int refine3f(const Geo& g, const Box& B, const Box3F& F, const float* Wg,
                                        const Seed* __restrict__ seeds, double beta, int nrhs, double tol,
                                        int max_refine, Gj3f& sm, float wc[JC][R3], double& omega) {
  int it = 1;
  while (true) {
    omega = resid3f<NW>(g, B, F, seeds, beta, nrhs, sm);
    if (omega <= tol) break;
    if (it > max_refine || !(omega <= 1e300)) {
      if (threadIdx.x == 0) atomicOr(&sm.flag, kFlagNoConv);
      break;
    }
    solve3f<NW, JCN>(F, wc, Wg, nrhs);
    update3f<NW>(F, nrhs);
    ++it;
  }
  return it;
}

__device__ __forceinline__ void record3f(int it, double omega, int* iters, unsigned long long* resid) {
  if (threadIdx.x == 0) {
    atomicMax(iters, it);
    atomicMax(resid, (unsigned long long)__double_as_longlong(omega));
  }
}

// Xf = D^-1/2 b for x = 0 (b in X, or in Bv when FROM_BV), and X = 0.
template <int NW, bool FROM_BV>
__device__ __forceinline__ void start3f(const Box3F& F, int nrhs) {
  const int nc = F.s.nc;
  for (int e = threadIdx.x; e < nrhs * nc; e += 64 * NW) {
    const int loc = e % nc;
    const double b = FROM_BV ? F.Bv[loc] : F.s.X[e];
    F.Xf[e] = (float)(F.sd[loc] * b);
    F.s.X[e] = 0.0;
  }
  bsync<NW>();
}

// Steps 1-2 on an oversampled box (FO: Step 6, the factor alone).
template <int NW, bool FO, bool TS>
__device__ __forceinline__ void basis3f(const Geo& g, const Box& B, const Seed* __restrict__ seeds,
                                        const double* __restrict__ logK, double beta, float* __restrict__ fac,
                                        double* __restrict__ Pk, double* __restrict__ tr_u,
                                        double* __restrict__ tr_phi, double* __restrict__ tr_beta,
                                        double tol, int max_refine, int* iters, unsigned long long* resid,
                                        double* dsm, Gj3f& sm) {
  constexpr int NT = 64 * NW;
  const int nrhs = FO ? 0 : B.nrhs;
  // the seeds in batches of at most kSeedBatch3f (the LDS of one batch's
  // FP64 solutions and FP32 work vectors), after the factor
  const int nbat = nrhs < kSeedBatch3f ? nrhs : kSeedBatch3f;
  Box3F F = carve3f<TS>(dsm, B, nbat, 0, g.kc);
  Box3& s = F.s;
  load_box3<NW, true>(g, B, logK, beta, s);
  scale3f<NW>(F);
  float* Wg = fac + B.fac;
  float wc[JC][R3];
  factor3f<NW, 0>(g, B, F, Wg, 0, sm, wc);
  if (FO) return;
  // the first JCB planes' inverses as row blocks in registers (a forward
  // sweep fused with the factor needs more registers than three boxes per
  // CU leave, and was slower); the barrier orders the last plane's stores
  // before the reads of other waves
  bsync<NW>();
  const int nb = s.m0 * s.m1;
#pragma unroll
  for (int j = 0; j < JCB; ++j)
    if (j < s.m2) load_rb(Wg + (long long)j * nb * nb, nb, wc[j]);
  for (int b0 = 0; b0 < nrhs; b0 += kSeedBatch3f) {
    const int nr = min(kSeedBatch3f, nrhs - b0);
    Box Bb = B;  // seeds b0 .. b0 + nr - 1
    Bb.seed0 += b0;
    for (int e = threadIdx.x; e < nr * s.nc; e += NT) s.X[e] = 0.0;
    bsync<NW>();
    seed_rhs3<NW>(g, Bb, s, seeds, beta, nr, s.X);
    bsync<NW>();
    start3f<NW, false>(F, nr);
    solve3f<NW, JCB>(F, wc, Wg, nr);
    update3f<NW>(F, nr);
    double omega;
    const int it = refine3f<NW, JCB>(g, Bb, F, Wg, seeds, beta, nr, tol, max_refine, sm, wc, omega);
    record3f(it, omega, iters, resid);
    basis_out3<NW>(g, Bb, s, seeds, beta, nr, Pk, tr_u, tr_phi, tr_beta);
    bsync<NW>();  // X is read by the outputs before the next batch clears it
  }
}

// Step 4 on a subdomain; writes K = exp(log K) of its cells.
template <int NW, bool TS>
__device__ __forceinline__ void particular3f(const Geo& g, const Box& B, const double* __restrict__ logK,
                                             double* __restrict__ K, const double* __restrict__ f,
                                             const double* __restrict__ bcv, double beta,
                                             float* __restrict__ fac, double* __restrict__ pbar,
                                             double* __restrict__ ubar, double* __restrict__ pibar,
                                             double tol, int max_refine, int* iters,
                                             unsigned long long* resid, double* dsm, Gj3f& sm) {
  Box3F F = carve3f<TS>(dsm, B, 1, 1, g.kc);
  Box3& s = F.s;
  load_box3<NW, true>(g, B, logK, beta, s);
  part_k3<NW, TS>(g, B, s, K, sm.flag);
  physical3<NW>(g, B, s, f, bcv, F.Bv);
  scale3f<NW>(F);
  start3f<NW, true>(F, 1);
  stage0_rb<NW>(rbv(F, 1), s.m0 * s.m1);
  float* Wg = fac + B.fac;
  float wc[JC][R3];  // not used: a subdomain's few small planes are read back
  factor3f<NW, 0>(g, B, F, Wg, 1, sm, wc);
  backward3f<NW, 0>(F, wc, Wg, 1);
  update3f<NW>(F, 1);
  double omega;
  const int it = refine3f<NW, 0>(g, B, F, Wg, nullptr, beta, 1, tol, max_refine, sm, wc, omega);
  record3f(it, omega, iters, resid);
  part_out3<NW>(g, B, s, beta, pbar, ubar, pibar);
}

// Steps 6-7 for one box: right-hand side from the state, FP32 solves with
// the stored inverses (read once into the register cache), FP64
// refinement, then p on Omega_i and Omega_i's Gamma fluxes.
template <int NW, bool TS, int JCN>
__device__ __forceinline__ void smooth3f(const Geo& g, const Box& B, const double* __restrict__ K,
                                         const double* __restrict__ f, const double* __restrict__ bcv,
                                         double beta, const float* __restrict__ fac, double* p,
                                         double* gflux, double tol, int max_refine, int* iters,
                                         unsigned long long* resid, double* dsm, Gj3f& sm) {
  Box3F F = carve3f<TS>(dsm, B, 1, 1, g.kc);
  Box3& s = F.s;
  load_box3<NW, false>(g, B, K, beta, s);
  physical3<NW>(g, B, s, f, bcv, F.Bv);
  bsync<NW>();
  smooth_rhs3<NW>(g, B, s, p, gflux, beta, F.Bv);
  scale3f<NW>(F);
  start3f<NW, true>(F, 1);
  stage0_rb<NW>(rbv(F, 1), s.m0 * s.m1);
  const float* Wg = fac + B.fac;
  float wc[JC][R3];
  forward3f<NW, true, JCN>(F, wc, Wg, 1);
  backward3f<NW, JCN>(F, wc, Wg, 1);
  update3f<NW>(F, 1);
  double omega;
  const int it = refine3f<NW, JCN>(g, B, F, Wg, nullptr, beta, 1, tol, max_refine, sm, wc, omega);
  record3f(it, omega, iters, resid);
  smooth_out3<NW>(g, B, s, p, gflux, beta);
}

// Three boxes per CU (LDS of an 8 x 8 x 8 basis box with a batch of three
// seeds about 48 KB with its pivot buffers): up to 168 registers per lane.
template <int NW, bool TS>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3)))
k_basis3f(Geo g, const Box* __restrict__ boxes, const Seed* __restrict__ seeds, const double* __restrict__ logK,
          double beta, float* __restrict__ fac, double* __restrict__ Pk, double* __restrict__ tr_u,
          double* __restrict__ tr_phi, double* __restrict__ tr_beta, int factor_only, double tol,
          int max_refine, int* iters, unsigned long long* resid, int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ Gj3f sm;
  if (threadIdx.x == 0) sm.flag = 0;
  bsync<NW>();
  const Box B = boxes[blockIdx.x];
  if (factor_only)
    basis3f<NW, true, TS>(g, B, seeds, logK, beta, fac, Pk, tr_u, tr_phi, tr_beta, tol, max_refine, iters,
                          resid, dsm, sm);
  else
    basis3f<NW, false, TS>(g, B, seeds, logK, beta, fac, Pk, tr_u, tr_phi, tr_beta, tol, max_refine, iters,
                           resid, dsm, sm);
  bsync<NW>();
  if (threadIdx.x == 0 && sm.flag) atomicOr(flags, sm.flag);
}

template <int NW, bool TS>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2)))
k_particular3f(Geo g, const Box* __restrict__ boxes, const double* __restrict__ logK, double* __restrict__ K,
               const double* __restrict__ f, const double* __restrict__ bcv, double beta,
               float* __restrict__ fac, double* __restrict__ pbar, double* __restrict__ ubar,
               double* __restrict__ pibar, double tol, int max_refine, int* iters, unsigned long long* resid,
               int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ Gj3f sm;
  if (threadIdx.x == 0) sm.flag = 0;
  bsync<NW>();
  const Box B = boxes[blockIdx.x];
  particular3f<NW, TS>(g, B, logK, K, f, bcv, beta, fac, pbar, ubar, pibar, tol, max_refine, iters, resid,
                       dsm, sm);
  bsync<NW>();
  if (threadIdx.x == 0 && sm.flag) atomicOr(flags, sm.flag);
}

// JCN planes' inverses held in registers across the refinement sweeps, the
// others read from memory by every sweep: JCN = 8 (two boxes per CU), 4
// (three), 2 or 0 (four; LDS of an 8 x 8 x 8 smoothing box about 33 KB).
template <int NW, bool TS, int JCN>
__global__ void __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(JCN == JC ? 2 : JCN > 2 ? 3 : 4)))
k_smooth3f(Geo g, const Box* __restrict__ boxes, const double* __restrict__ K, const double* __restrict__ f,
           const double* __restrict__ bcv, double beta, const float* __restrict__ fac, double* __restrict__ p,
           double* __restrict__ gflux, double tol, int max_refine, int* iters, unsigned long long* resid,
           int* flags) {
  extern __shared__ __align__(16) double dsm[];
  __shared__ Gj3f sm;
  if (threadIdx.x == 0) sm.flag = 0;
  bsync<NW>();
  const Box B = boxes[blockIdx.x];
  smooth3f<NW, TS, JCN>(g, B, K, f, bcv, beta, fac, p, gflux, tol, max_refine, iters, resid, dsm, sm);
  bsync<NW>();
  if (threadIdx.x == 0 && sm.flag) atomicOr(flags, sm.flag);
}

template <typename KF>
hipError_t lds_attr3f(KF kern, size_t bytes) {
  if (bytes > 64 * 1024)
    return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return hipSuccess;
}

}  // namespace

size_t box3f_lds_bytes(int m0, int m1, int m2, int nrhs, int nbv, int kc) {
  return box3f_bytes(m0, m1, m2, nrhs, nbv, kc);
}

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

hipError_t launch_basis3f(const Geo& g, const Box* boxes, int nbox, const Seed* seeds, const double* logK,
                          double beta, float* fac32, double* Pk, double* tr_u, double* tr_phi,
                          double* tr_beta, int factor_only, double tol, int max_refine, int* iters,
                          unsigned long long* resid, int* flags, size_t lds, int nw, hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
#define MRCM_CALL(NW, TS)                                                                                   \
  e = lds_attr3f(k_basis3f<NW, TS>, lds);                                                                   \
  if (e != hipSuccess) return e;                                                                            \
  hipLaunchKernelGGL((k_basis3f<NW, TS>), dim3(nbox), dim3(64 * NW), lds, s, g, boxes, seeds, logK, beta,   \
                     fac32, Pk, tr_u, tr_phi, tr_beta, factor_only, tol, max_refine, iters, resid, flags)
  MRCM_NW_SWITCH(nw, MRCM_CALL)
#undef MRCM_CALL
  return hipGetLastError();
}

hipError_t launch_particular3f(const Geo& g, const Box* boxes, int nbox, const double* logK, double* K,
                               const double* f, const double* bcv, double beta, float* facp32,
                               double* pbar, double* ubar, double* pibar, double tol, int max_refine,
                               int* iters, unsigned long long* resid, int* flags, size_t lds, int nw,
                               hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
#define MRCM_CALL(NW, TS)                                                                                   \
  e = lds_attr3f(k_particular3f<NW, TS>, lds);                                                              \
  if (e != hipSuccess) return e;                                                                            \
  hipLaunchKernelGGL((k_particular3f<NW, TS>), dim3(nbox), dim3(64 * NW), lds, s, g, boxes, logK, K, f,     \
                     bcv, beta, facp32, pbar, ubar, pibar, tol, max_refine, iters, resid, flags)
  MRCM_NW_SWITCH(nw, MRCM_CALL)
#undef MRCM_CALL
  return hipGetLastError();
}

hipError_t launch_smooth3f(const Geo& g, const Box* boxes, int nmem, const double* K, const double* f,
                           const double* bcv, double beta, const float* fac32, double* p, double* gflux,
                           double tol, int max_refine, int* iters, unsigned long long* resid, int* flags,
                           size_t lds, int nw, int cached, hipStream_t s) {
  if (nmem <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
#define MRCM_CALL1(NW, TS, JCN)                                                                             \
  e = lds_attr3f(k_smooth3f<NW, TS, JCN>, lds);                                                             \
  if (e != hipSuccess) return e;                                                                            \
  hipLaunchKernelGGL((k_smooth3f<NW, TS, JCN>), dim3(nmem), dim3(64 * NW), lds, s, g, boxes, K, f, bcv,     \
                     beta, fac32, p, gflux, tol, max_refine, iters, resid, flags)
#define MRCM_CALL(NW, TS)          \
  if (cached >= JC) {              \
    MRCM_CALL1(NW, TS, JC);        \
  } else if (cached >= 4) {        \
    MRCM_CALL1(NW, TS, 4);         \
  } else if (cached > 0) {         \
    MRCM_CALL1(NW, TS, 2);         \
  } else {                         \
    MRCM_CALL1(NW, TS, 0);         \
  }
  MRCM_NW_SWITCH(nw, MRCM_CALL)
#undef MRCM_CALL
#undef MRCM_CALL1
  return hipGetLastError();
}

#undef MRCM_NW_SWITCH

}  // namespace mrcm
