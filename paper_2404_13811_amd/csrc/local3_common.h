// Device code shared by the 3-D local kernels of the two precision forms
// (FP64 in local3.hip; FP32 factors with FP64 refinement in local3f.hip):
// the LDS layout of a box (K tile with a one-cell halo, diagonal, couplings
// to the next plane, solution vectors), the assembly of its two-point-flux
// matrix, the geometry of subdomains, seeds and faces, the right-hand
// sides of the physical data and of the smoothing Robin data (Section 3),
// and the outputs of Steps 1-2, 4 and 7 from a box's solution.
#pragma once
#include "local_common.h"

namespace mrcm {
namespace {

constexpr int P3 = 64;   // lanes: columns of the padded plane block
constexpr int R3 = 16;   // rows of the block per lane
constexpr int G3 = 4;    // pivots per Gauss-Jordan step

__device__ __forceinline__ int lane3() { return threadIdx.x & 63; }

// The lane index recomputed where it is used: the unrolled elimination
// steps would otherwise each get lane-dependent constants (pivot-column
// masks, unit right-hand sides) computed up front and kept in scratch
// memory for the whole elimination.
__device__ __forceinline__ int lane3_here() {
  int v;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(v));
  return v;
}
// wave index as a scalar, so that branches on it are uniform
__device__ __forceinline__ int wave3() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// LDS ordering between the lanes of the box: within one wave a wait for the
// LDS counter is enough; several waves meet at the workgroup barrier.
template <int NW>
__device__ __forceinline__ void bsync() {
  if constexpr (NW == 1) {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// The same for steps whose exchange between waves is LDS only (the sweep
// steps): the fences order LDS accesses alone, so global loads issued
// ahead (the next plane's inverse) stay in flight across the barrier.
template <int NW>
__device__ __forceinline__ void lsync() {
  if constexpr (NW == 1) {
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  }
}

// Row-block sweeps (both precision forms).  A second register layout of a
// plane inverse: lane L of wave v holds W_j[r][16q .. 16q + 15] with
// r = 16v + L / 4 and q = L % 4, so y_r = (W_j z)_r is a 16-term dot
// product per lane summed over the four lanes of a quad (DPP), with no
// exchange between waves.  Each step of a sweep reads the plane's staged
// input vector from LDS, writes y into the solution vectors and stages the
// next plane's input, then meets the other waves at one barrier (LDS
// only).  Rows and columns beyond the nb x nb block hold 0.
__device__ __forceinline__ int rb_row() { return R3 * wave3() + (lane3() >> 2); }
__device__ __forceinline__ int rb_col() { return R3 * (lane3() & 3); }

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

// sum over the quad: quad_perm(1,0,3,2) then quad_perm(2,3,0,1); every
// lane of the quad gets the same value
__device__ __forceinline__ float quad_sum(float p) {
  p += __int_as_float(dpp_i<0xB1>(__float_as_int(p)));
  p += __int_as_float(dpp_i<0x4E>(__float_as_int(p)));
  return p;
}

__device__ __forceinline__ double quad_sum(double p) {
  p += __hiloint2double(dpp_i<0xB1>(__double2hiint(p)), dpp_i<0xB1>(__double2loint(p)));
  p += __hiloint2double(dpp_i<0x4E>(__double2hiint(p)), dpp_i<0x4E>(__double2loint(p)));
  return p;
}

// 16-byte loads of four floats or two doubles
template <typename T>
__device__ __forceinline__ void ld16(const T* src, T* dst) {
  if constexpr (sizeof(T) == 4) {
    const float4 v = *reinterpret_cast<const float4*>(src);
    dst[0] = v.x;
    dst[1] = v.y;
    dst[2] = v.z;
    dst[3] = v.w;
  } else {
    const double2 v = *reinterpret_cast<const double2*>(src);
    dst[0] = v.x;
    dst[1] = v.y;
  }
}

// The lane's row-block entries of a stored inverse (nb x nb, row-major).
template <typename T>
__device__ __forceinline__ void load_rb(const T* Wj, int nb, T wr[R3]) {
  constexpr int V = 16 / sizeof(T);
  const int r = rb_row(), c0 = rb_col();
  const T* src = Wj + r * nb + c0;
  if (r < nb && c0 + R3 <= nb && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
#pragma unroll
    for (int ii = 0; ii < R3; ii += V) ld16(src + ii, wr + ii);
  } else {
#pragma unroll
    for (int ii = 0; ii < R3; ++ii) wr[ii] = (r < nb && c0 + ii < nb) ? src[ii] : T(0);
  }
}

template <typename T>
__device__ __forceinline__ T dot16(const T wr[R3], const T* z) {
  constexpr int V = 16 / sizeof(T);
  T a0 = T(0), a1 = T(0);
#pragma unroll
  for (int ii = 0; ii < R3; ii += V) {
    T zz[V];
    ld16(z + ii, zz);
#pragma unroll
    for (int u = 0; u < V; u += 2) {
      a0 = fma(wr[ii + u], zz[u], a0);
      a1 = fma(wr[ii + u + 1], zz[u + 1], a1);
    }
  }
  return a0 + a1;
}

// The vectors a row-block sweep works on: X (nrhs x nc, solved in place),
// the plane couplings Tz (ncell) and the staged inputs Z (2 x nrhs x 64,
// 16-byte aligned).
template <typename T>
struct RbSweep {
  T* X;
  const T* Tz;
  T* Z;
  int nc, m2, nrhs;
};

// Staged inputs of plane j: two alternating buffers; a step reads one and
// writes the other.
template <typename T>
__device__ __forceinline__ T* zbuf(const RbSweep<T>& v, int j) { return v.Z + (j & 1) * v.nrhs * P3; }

// Input of plane 0 of a forward sweep from X (the right-hand sides).
template <int NW, typename T>
__device__ __forceinline__ void stage0_rb(const RbSweep<T>& v, int nb) {
  for (int e = threadIdx.x; e < v.nrhs * P3; e += 64 * NW) {
    const int k = e / P3, i = e % P3;
    v.Z[e] = i < nb ? v.X[k * v.nc + i] : T(0);
  }
  lsync<NW>();
}

// Forward step of plane j: z_j = W_j (r_j + t_{j-1} z_{j-1}) into X, and
// the next plane's input r_{j+1} + t_j z_j, or on the last plane the input
// t_{j-1} x_j of the backward sweep's first plane (x_j = z_j there).
template <int NW, typename T>
__device__ __forceinline__ void fwd_rb(const RbSweep<T>& v, int nb, int j, const T wr[R3]) {
  const int r = rb_row(), c0 = rb_col(), nc = v.nc;
  const bool last = j == v.m2 - 1;
  const T* zin = zbuf(v, j);
  T* zout = zbuf(v, j + 1);
  for (int k = 0; k < v.nrhs; ++k) {
    T y = c0 < nb ? dot16(wr, zin + k * P3 + c0) : T(0);
    y = quad_sum(y);
    if (c0 == 0) {
      T zn = T(0);
      if (r < nb) {
        v.X[k * nc + j * nb + r] = y;
        if (!last) zn = fma(v.Tz[j * nb + r], y, v.X[k * nc + (j + 1) * nb + r]);
        else if (j > 0) zn = v.Tz[(j - 1) * nb + r] * y;
      }
      zout[k * P3 + r] = zn;
    }
  }
  lsync<NW>();
}

// Backward step of plane j: x_j = z_j + W_j (t_j .* x_{j+1}) into X, and
// the input t_{j-1} x_j of plane j - 1.
template <int NW, typename T>
__device__ __forceinline__ void bwd_rb(const RbSweep<T>& v, int nb, int j, const T wr[R3]) {
  const int r = rb_row(), c0 = rb_col(), nc = v.nc;
  const T* zin = zbuf(v, j);
  T* zout = zbuf(v, j + 1);
  for (int k = 0; k < v.nrhs; ++k) {
    T y = c0 < nb ? dot16(wr, zin + k * P3 + c0) : T(0);
    y = quad_sum(y);
    if (c0 == 0) {
      T zn = T(0);
      if (r < nb) {
        const T x = v.X[k * nc + j * nb + r] + y;
        v.X[k * nc + j * nb + r] = x;
        if (j > 0) zn = v.Tz[(j - 1) * nb + r] * x;
      }
      zout[k * P3 + r] = zn;
    }
  }
  lsync<NW>();
}

// LDS of one box.
struct Box3 {
  double* Kt;  // (m0 + 2)(m1 + 2)(m2 + 2) permeabilities, one-cell halo
  double* Dg;  // ncell diagonal
  double* Tz;  // ncell coupling to the next plane (0 on the last plane)
  double* X;   // nrhs x ncell right-hand sides / solutions
  double* Z;   // nrhs x 64 staging of one block
  int m0, m1, m2, nc;
  // diagonal permeability tensor: halo tiles of the entries of axes 1..,
  // ktn doubles apart (ktn = 0: scalar K), and the tile each axis reads
  // (Kt for every axis with scalar K)
  double* Kx;
  int ktn;
  const double* Ka[2];  // axes 1 and 2
};

// LDS of those extra tiles (ahead of the box's other arrays; even).
__host__ __device__ inline size_t kx3_doubles(int kc, int m0, int m1, int m2) {
  return kc > 1 ? ((size_t)(kc - 1) * (m0 + 2) * (m1 + 2) * (m2 + 2) + 1) / 2 * 2 : 0;
}

__host__ __device__ inline size_t box3_doubles(int m0, int m1, int m2, int nrhs, int kc = 1) {
  const size_t nc = (size_t)m0 * m1 * m2;
  return kx3_doubles(kc, m0, m1, m2) + (size_t)(m0 + 2) * (m1 + 2) * (m2 + 2) + 2 * nc +
         (size_t)nrhs * nc + (size_t)nrhs * P3 + 4;
}

// TS: the tensor form; without it the tiles of axes 1.. are Kt at
// compile time, and the scalar kernels carry nothing of the tensor.
template <bool TS>
__device__ __forceinline__ Box3 carve3(double* base, const Box& B, int nrhs, int kc) {
  if (!TS) kc = 1;
  Box3 s;
  s.m0 = B.hi[0] - B.lo[0];
  s.m1 = B.hi[1] - B.lo[1];
  s.m2 = B.hi[2] - B.lo[2];
  s.nc = s.m0 * s.m1 * s.m2;
  s.Kx = base;
  s.ktn = kc > 1 ? (s.m0 + 2) * (s.m1 + 2) * (s.m2 + 2) : 0;
  base += kx3_doubles(kc, s.m0, s.m1, s.m2);
  s.Kt = base;
  s.Ka[0] = s.ktn ? s.Kx : s.Kt;
  s.Ka[1] = s.ktn ? s.Kx + s.ktn : s.Kt;
  s.Dg = s.Kt + (s.m0 + 2) * (s.m1 + 2) * (s.m2 + 2);
  s.Tz = s.Dg + s.nc;
  s.X = s.Tz + s.nc;
  double* z = s.X + (size_t)nrhs * s.nc;
  // 16-byte alignment for the paired reads of Z
  const long long off = z - base;
  s.Z = base + ((off + 1) & ~1LL);
  return s;
}

// K along axis a at global cell (x, y, z) of the box or its halo.
__device__ __forceinline__ double k3(const Box3& s, const Box& B, int x, int y, int z, int a) {
  // a select of the pointer values, not of the fields' addresses (that
  // would keep the fields in scratch memory)
  const double *t0 = s.Kt, *t1 = s.Ka[0], *t2 = s.Ka[1];
  const double* t = a == 0 ? t0 : a == 1 ? t1 : t2;
  return t[((z - B.lo[2] + 1) * (s.m1 + 2) + (y - B.lo[1] + 1)) * (s.m0 + 2) + (x - B.lo[0] + 1)];
}

__device__ __forceinline__ double rcp3(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// K tile (log K when LOG: exponentiated here) and the diagonal and plane
// couplings of the box matrix.
template <int NW, bool LOG>
__device__ __forceinline__ void load_box3(const Geo& g, const Box& B, const double* Kg, double beta,
                                          Box3& s) {
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x;
  const int W0 = s.m0 + 2, W1 = s.m1 + 2, W2 = s.m2 + 2;
  const int nt = W0 * W1 * W2;
  for (int e0 = 0; e0 < nt; e0 += NT * 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * NT + tid;
      const int x = B.lo[0] - 1 + e % W0, y = B.lo[1] - 1 + (e / W0) % W1, z = B.lo[2] - 1 + e / (W0 * W1);
      const bool in = e < nt && x >= 0 && x < g.n[0] && y >= 0 && y < g.n[1] && z >= 0 && z < g.n[2];
      v[u] = in ? Kg[x + g.n[0] * (y + g.n[1] * z)] : (LOG ? 0.0 : 1.0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * NT + tid;
      if (e < nt) s.Kt[e] = LOG ? exp(v[u]) : v[u];
    }
  }
  // the other axes' entries of a diagonal tensor
  for (int e = tid; e < (s.ktn ? (g.kc - 1) * nt : 0); e += NT) {
    const int ax = 1 + e / nt, u = e - (ax - 1) * nt;
    const int x = B.lo[0] - 1 + u % W0, y = B.lo[1] - 1 + (u / W0) % W1, z = B.lo[2] - 1 + u / (W0 * W1);
    const bool in = x >= 0 && x < g.n[0] && y >= 0 && y < g.n[1] && z >= 0 && z < g.n[2];
    const double v = in ? Kg[kaxis(g, ax) + x + g.n[0] * (y + g.n[1] * z)] : (LOG ? 0.0 : 1.0);
    s.Kx[e] = LOG ? exp(v) : v;
  }
  bsync<NW>();
  const double ih = rcp3(g.h);
  for (int loc = tid; loc < s.nc; loc += NT) {
    const int x = B.lo[0] + loc % s.m0, y = B.lo[1] + (loc / s.m0) % s.m1, z = B.lo[2] + loc / (s.m0 * s.m1);
    double diag = 0.0, tz = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double kc = k3(s, B, x, y, z, a);
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        int o[3] = {x, y, z};
        o[a] += sd ? 1 : -1;
        if (o[a] < 0 || o[a] >= g.n[a]) {
          if (g.bc_type[2 * a + sd]) diag += 2.0 * kc * g.area * ih;
          continue;
        }
        const double ko = k3(s, B, o[0], o[1], o[2], a);
        const bool inside = o[a] >= B.lo[a] && o[a] < B.hi[a];
        if (inside) {
          const double T = g.area * 2.0 * kc * ko * rcp3(kc + ko) * ih;
          diag += T;
          if (a == 2 && sd) tz = T;
        } else {
          const double bt = robin_beta(g, a, kc, ko, beta);
          diag += robin_T(g, kc, bt);
        }
      }
    }
    s.Dg[loc] = diag;
    s.Tz[loc] = tz;
  }
  bsync<NW>();
}

// In-plane coupling between plane cells a and a + dx (dx = 1: x, m0: y) of
// plane j, from the K tile (0 when the neighbour is outside the box).
__device__ __forceinline__ double tplane(const Geo& g, const Box& B, const Box3& s, int j, int a, int axis) {
  const int x = B.lo[0] + a % s.m0, y = B.lo[1] + a / s.m0, z = B.lo[2] + j;
  const int ox = x + (axis == 0), oy = y + (axis == 1);
  if (ox >= B.hi[0] || oy >= B.hi[1]) return 0.0;
  const double kc = k3(s, B, x, y, z, axis), ko = k3(s, B, ox, oy, z, axis);
  return g.area * 2.0 * kc * ko * rcp3(kc + ko) * rcp3(g.h);
}

__device__ __forceinline__ int bloc3(const Box& B, const Box3& s, const int c[3]) {
  return (c[0] - B.lo[0]) + s.m0 * ((c[1] - B.lo[1]) + s.m1 * (c[2] - B.lo[2]));
}

__device__ __forceinline__ void omega3(const Geo& g, int sub, int lo[3], int hi[3]) {
  int r = sub;
  for (int a = 0; a < 3; ++a) {
    const int ia = r % g.M[a];
    r /= g.M[a];
    lo[a] = ia * g.S[a];
    hi[a] = lo[a] + g.S[a];
  }
}

__device__ __forceinline__ int nbr3(const Geo& g, int sub, int q) {
  const int a = q >> 1, sd = q & 1;
  int stride = 1;
  for (int b = 0; b < a; ++b) stride *= g.M[b];
  const int ia = (sub / stride) % g.M[a];
  const int t = ia + (sd ? 1 : -1);
  if (t < 0 || t >= g.M[a]) return -1;
  return sub + (sd ? stride : -stride);
}

__device__ __forceinline__ void face3(const int lo[3], const int hi[3], int q, int t, int c[3]) {
  const int a = q >> 1, sd = q & 1;
  int r = t;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    if (b == a) {
      c[b] = sd ? hi[b] - 1 : lo[b];
    } else {
      const int m = hi[b] - lo[b];
      c[b] = lo[b] + r % m;
      r /= m;
    }
  }
}

__device__ __forceinline__ bool inbox3(const Box& B, const int c[3]) {
  return c[0] >= B.lo[0] && c[0] < B.hi[0] && c[1] >= B.lo[1] && c[1] < B.hi[1] && c[2] >= B.lo[2] &&
         c[2] < B.hi[2];
}

// Right-hand side of the physical data (source, boundary conditions).
template <int NW>
__device__ __forceinline__ void physical3(const Geo& g, const Box& B, const Box3& s,
                                          const double* __restrict__ f,
                                          const double* __restrict__ bcv, double* X) {
  for (int loc = threadIdx.x; loc < s.nc; loc += 64 * NW) {
    const int c[3] = {B.lo[0] + loc % s.m0, B.lo[1] + (loc / s.m0) % s.m1, B.lo[2] + loc / (s.m0 * s.m1)};
    const int ci = gcell(g, c);
    double b = f[ci] * g.vol;
    for (int a = 0; a < 3; ++a)
      for (int sd = 0; sd < 2; ++sd) {
        const int t = c[a] + (sd ? 1 : -1);
        if (t >= 0 && t < g.n[a]) continue;
        const int side = 2 * a + sd;
        const double val = bcv[g.bc_off[side] + bface_index(g, c, a)];
        if (g.bc_type[side]) b += 2.0 * k3(s, B, c[0], c[1], c[2], a) * g.area / g.h * val;
        else b -= g.area * val;
      }
    X[loc] = b;
  }
}

// Robin data lambda on face (a, sd) of box cell c from the current state
// (Section 3 item 3): from the two-point flux across the face when the
// outside cell lies in the neighbouring subdomain's reach (overlap > 0), or
// from the neighbour's own Gamma flux and trace (overlap 0).
__device__ __forceinline__ double lambda3(const Geo& g, const Box& B, const Box3& s,
                                          const double* __restrict__ p,
                                          const double* __restrict__ gflux, double beta,
                                          const int c[3], int a, int sd) {
  int o[3] = {c[0], c[1], c[2]};
  o[a] += sd ? 1 : -1;
  const double kc = k3(s, B, c[0], c[1], c[2], a), ko = k3(s, B, o[0], o[1], o[2], a);
  const double bt = robin_beta(g, a, kc, ko, beta);
  const int ci = gcell(g, c), oi = gcell(g, o);
  if (g.l > 0) {
    const double u = g.area * kharm(kc, ko) / g.h * (p[ci] - p[oi]) / g.area;
    const double pi = p[ci] - u * g.h / (2.0 * kc);
    return -bt * u + pi;
  }
  const int q = 2 * a + sd;
  const int j = nbr3(g, B.sub, q);
  int jlo[3], jhi[3];
  omega3(g, j, jlo, jhi);
  const int t = side_face_index(g, jlo, jhi, o, a);
  const double uj = gflux[(long long)j * g.gstride + g.gside_off[q ^ 1] + t];
  const double pij = p[oi] - uj * g.h / (2.0 * ko);
  return bt * uj + pij;
}


// Right-hand side of a seed on box cell c of the seed's side: T^R times
// the seed's value on the face.
__device__ __forceinline__ double seed_face_b3(const Geo& g, const Box& B, const Box3& s, const Seed& sd,
                                               double beta, const int c[3]) {
  const int a = sd.side >> 1, d = (sd.side & 1) ? 1 : -1;
  const double kc = k3(s, B, c[0], c[1], c[2], a);
  const double ko = k3(s, B, c[0] + (a == 0 ? d : 0), c[1] + (a == 1 ? d : 0), c[2] + (a == 2 ? d : 0), a);
  return robin_T(g, kc, robin_beta(g, a, kc, ko, beta)) * seed_value(g, sd, B.lo, B.hi, c);
}

// The seeds' right-hand sides into X (nrhs x ncell, zero on entry): T^R
// times the seed on the cells of its side.
template <int NW>
__device__ __forceinline__ void seed_rhs3(const Geo& g, const Box& B, const Box3& s,
                                          const Seed* __restrict__ seeds, double beta, int nrhs,
                                          double* X) {
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x;
  for (int k = 0; k < nrhs; ++k) {
    const Seed sd = seeds[B.seed0 + k];
    const int a = sd.side >> 1;
    int nf = 1;
    for (int b = 0; b < 3; ++b)
      if (b != a) nf *= B.hi[b] - B.lo[b];
    for (int t = tid; t < nf; t += NT) {
      int c[3];
      face3(B.lo, B.hi, sd.side, t, c);
      X[k * s.nc + bloc3(B, s, c)] = seed_face_b3(g, B, s, sd, beta, c);
    }
  }
}

// Outputs of Steps 1-2 from the seeds' solutions in s.X: the basis
// functions restricted to Omega_i, and on Gamma_i the flux, the Robin datum
// phi = -beta u + pi and the Robin parameter of every face.
template <int NW>
__device__ __forceinline__ void basis_out3(const Geo& g, const Box& B, const Box3& s,
                                           const Seed* __restrict__ seeds, double beta, int nrhs,
                                           double* __restrict__ Pk, double* __restrict__ tr_u,
                                           double* __restrict__ tr_phi, double* __restrict__ tr_beta) {
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x;
  int olo[3], ohi[3];
  omega3(g, B.sub, olo, ohi);
  const int ncell_o = g.S[0] * g.S[1] * g.S[2];
  for (int e = tid; e < nrhs * ncell_o; e += NT) {
    const int k = e / ncell_o, t = e % ncell_o;
    const int c[3] = {olo[0] + t % g.S[0], olo[1] + (t / g.S[0]) % g.S[1], olo[2] + t / (g.S[0] * g.S[1])};
    Pk[(long long)(B.seed0 + k) * ncell_o + t] = s.X[k * s.nc + bloc3(B, s, c)];
  }
  for (int q = 0; q < 6; ++q) {
    const int a = q >> 1, so = q & 1;
    int nf = 1;
    for (int b = 0; b < 3; ++b)
      if (b != a) nf *= g.S[b];
    const bool has = nbr3(g, B.sub, q) >= 0;
    for (int e = tid; e < nrhs * nf; e += NT) {
      const int k = e / nf, t = e % nf;
      const long long oidx = (long long)(B.seed0 + k) * g.gstride + g.gside_off[q] + t;
      if (!has) {
        tr_u[oidx] = 0.0;
        tr_phi[oidx] = 0.0;
        continue;
      }
      int c[3];
      face3(olo, ohi, q, t, c);
      int o[3] = {c[0], c[1], c[2]};
      o[a] += so ? 1 : -1;
      const double kc = k3(s, B, c[0], c[1], c[2], a), ko = k3(s, B, o[0], o[1], o[2], a);
      const double Pc = s.X[k * s.nc + bloc3(B, s, c)];
      const double bt = robin_beta(g, a, kc, ko, beta);
      double u;
      if (inbox3(B, o)) {
        u = g.area * kharm(kc, ko) / g.h * (Pc - s.X[k * s.nc + bloc3(B, s, o)]) / g.area;
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
}

// K = exp(log K) of a subdomain's cells out to the global array (the
// subdomains cover the grid once); a K that is not finite and positive is
// flagged.
template <int NW, bool TS>
__device__ __forceinline__ void part_k3(const Geo& g, const Box& B, const Box3& s, double* __restrict__ K,
                                        int& flag) {
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x;
  for (int loc = tid; loc < s.nc; loc += NT) {
    const int c[3] = {B.lo[0] + loc % s.m0, B.lo[1] + (loc / s.m0) % s.m1, B.lo[2] + loc / (s.m0 * s.m1)};
    for (int a = 0; a < (TS ? g.kc : 1); ++a) {
      const double k = k3(s, B, c[0], c[1], c[2], a);
      if (!(k > 0.0) || !isfinite(k)) atomicOr(&flag, kFlagBadK);
      K[kaxis(g, a) + gcell(g, c)] = k;
    }
  }
}

// Outputs of Step 4 from the solution in s.X: p-bar on Omega_i, and on
// Gamma_i the flux u-bar and pi-bar = beta u-bar (zero Robin data there).
template <int NW>
__device__ __forceinline__ void part_out3(const Geo& g, const Box& B, const Box3& s, double beta,
                                          double* __restrict__ pbar, double* __restrict__ ubar,
                                          double* __restrict__ pibar) {
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x;
  for (int t = tid; t < s.nc; t += NT) pbar[(long long)B.sub * s.nc + t] = s.X[t];
  for (int q = 0; q < 6; ++q) {
    const int a = q >> 1, so = q & 1;
    int nf = 1;
    for (int b = 0; b < 3; ++b)
      if (b != a) nf *= g.S[b];
    const bool has = nbr3(g, B.sub, q) >= 0;
    for (int t = tid; t < nf; t += NT) {
      const long long oidx = (long long)B.sub * g.gstride + g.gside_off[q] + t;
      if (!has) {
        ubar[oidx] = 0.0;
        pibar[oidx] = 0.0;
        continue;
      }
      int c[3];
      face3(B.lo, B.hi, q, t, c);
      int o[3] = {c[0], c[1], c[2]};
      o[a] += so ? 1 : -1;
      const double kc = k3(s, B, c[0], c[1], c[2], a);
      const double bt = robin_beta(g, a, kc, k3(s, B, o[0], o[1], o[2], a), beta);
      const double u = robin_T(g, kc, bt) * s.X[bloc3(B, s, c)] / g.area;
      ubar[oidx] = u;
      pibar[oidx] = bt * u;
    }
  }
}

// The Robin terms of the smoothing right-hand side added to X: T^R lambda
// on every Robin face of the box, lambda from the current state.
template <int NW>
__device__ __forceinline__ void smooth_rhs3(const Geo& g, const Box& B, const Box3& s,
                                            const double* __restrict__ p,
                                            const double* __restrict__ gflux, double beta, double* X) {
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x;
  for (int loc = tid; loc < s.nc; loc += NT) {
    const int c[3] = {B.lo[0] + loc % s.m0, B.lo[1] + (loc / s.m0) % s.m1, B.lo[2] + loc / (s.m0 * s.m1)};
    double add = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int sd = 0; sd < 2; ++sd) {
        const int o = c[a] + (sd ? 1 : -1);
        if (o < 0 || o >= g.n[a] || (o >= B.lo[a] && o < B.hi[a])) continue;
        int oc[3] = {c[0], c[1], c[2]};
        oc[a] = o;
        const double kc = k3(s, B, c[0], c[1], c[2], a);
        const double bt = robin_beta(g, a, kc, k3(s, B, oc[0], oc[1], oc[2], a), beta);
        add += robin_T(g, kc, bt) * lambda3(g, B, s, p, gflux, beta, c, a, sd);
      }
    X[loc] += add;
  }
}

// Outputs of Step 7 from the box solution in s.X: Omega_i's Gamma fluxes,
// then p on Omega_i.
template <int NW>
__device__ __forceinline__ void smooth_out3(const Geo& g, const Box& B, const Box3& s, double* p,
                                            double* gflux, double beta) {
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x;
  // Gamma fluxes of Omega_i (before p changes: with overlap 0 they read lambda)
  int olo[3], ohi[3];
  omega3(g, B.sub, olo, ohi);
  for (int q = 0; q < 6; ++q) {
    if (nbr3(g, B.sub, q) < 0) continue;
    const int a = q >> 1, sd = q & 1;
    int nf = 1;
    for (int b = 0; b < 3; ++b)
      if (b != a) nf *= g.S[b];
    for (int t = tid; t < nf; t += NT) {
      int c[3];
      face3(olo, ohi, q, t, c);
      int o[3] = {c[0], c[1], c[2]};
      o[a] += sd ? 1 : -1;
      const double kc = k3(s, B, c[0], c[1], c[2], a), ko = k3(s, B, o[0], o[1], o[2], a);
      const double xc = s.X[bloc3(B, s, c)];
      double u;
      if (inbox3(B, o)) {
        u = g.area * kharm(kc, ko) / g.h * (xc - s.X[bloc3(B, s, o)]) / g.area;
      } else {
        const double lam = lambda3(g, B, s, p, gflux, beta, c, a, sd);
        u = robin_T(g, kc, robin_beta(g, a, kc, ko, beta)) * (xc - lam) / g.area;
      }
      gflux[(long long)B.sub * g.gstride + g.gside_off[q] + t] = u;
    }
  }
  // every Robin datum of the box has been read before p is written
  bsync<NW>();
  const int ncell_o = g.S[0] * g.S[1] * g.S[2];
  for (int t = tid; t < ncell_o; t += NT) {
    const int c[3] = {olo[0] + t % g.S[0], olo[1] + (t / g.S[0]) % g.S[1], olo[2] + t / (g.S[0] * g.S[1])};
    p[gcell(g, c)] = s.X[bloc3(B, s, c)];
  }
}

}  // namespace
}  // namespace mrcm
