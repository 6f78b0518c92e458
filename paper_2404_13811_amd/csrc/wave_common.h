// Shared pieces of the one-wavefront-per-box 2-D local kernels (FP64 and
// FP32-with-refinement forms): LDS layout of a box, coefficient loading,
// the Gauss-Jordan block inverse in the two-half-wave register layout, and
// geometry helpers.  See local_wave.hip for the algorithm.
#pragma once
#include "local_common.h"
#include "pivot4.h"

namespace mrcm {
namespace wave {

constexpr int NBW = 32;
constexpr int HB = 16;
constexpr int RING = 4;

constexpr int GJB = 4;  // pivots per Gauss-Jordan step (one 4 x 4 pivot block)

// Pivot rows and columns of one Gauss-Jordan step (two alternating buffers):
// rowb[c * GJB + m] = A[k + m][c], colb[m * NBW + r] = A[r][k + m].
template <typename T>
struct __align__(16) GjSmem {
  T rowb[2][NBW * GJB];
  T colb[2][GJB * NBW];
  int flag;
};
using WaveSmem = GjSmem<double>;

// Dynamic LDS carve-up of one box.
struct BoxLds {
  double* Kt;   // (m0 + 2) x (m1 + 2) permeabilities, one-cell halo
  double* Dg;   // ncell diagonal of A
  double* Tx;   // ncell coupling to the x+1 neighbour (0 at the box edge)
  double* Tn;   // ncell coupling to the next block (y+1)
  double* X;    // nrhs x ncell right-hand sides / solutions
  double* Z;    // nrhs x NBW staging of one block
  int m0, m1;
  // diagonal permeability tensor: the halo tiles of the entries of axes
  // 1.., ktn doubles apart (ktn = 0: scalar K), and the tile axis 1 reads
  // (Kt with scalar K)
  double* Kx;
  int ktn;
  const double* Ky;
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// p rounded up to a 16-byte boundary (for 128-bit LDS accesses), measured
// from a 16-byte aligned base of the same array, so that the pointer keeps
// its address space.
template <typename T, typename B>
__device__ __forceinline__ T* align16(B* base, T* p) {
  constexpr int q = 16 / sizeof(T);
  const char* b = reinterpret_cast<const char*>(base);
  const long long off = (reinterpret_cast<const char*>(p) - b) / (long long)sizeof(T);
  return reinterpret_cast<T*>(const_cast<char*>(b)) + ((off + q - 1) / q) * q;
}

// Single-wave synchronisation through LDS: wait for this wave's LDS
// operations; the wave barrier keeps the compiler from moving memory
// operations across it.
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0) only
  __builtin_amdgcn_wave_barrier();
}

// Synchronisation of the NT threads working on one box (NT = 64: one wave).
template <int NT>
__device__ __forceinline__ void bsync() {
  if (NT == 64) wsync();
  else __syncthreads();
}

__device__ __forceinline__ double half_swap(double v) { return __shfl_xor(v, 32); }

// v(lane c) + v(lane c + 32) in every lane of column c, by two half-wave
// swaps of the 32-bit words (no LDS); both halves add in the same order.
__device__ __forceinline__ double half_sum(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}

__device__ __forceinline__ float half_sum_f(float v) {
  const int u = __float_as_int(v);
  const auto a = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  return __int_as_float(a[0]) + __int_as_float(a[1]);
}

// Cached block inverses of one box read through a buffer resource: per lane
// the byte offsets of its 16 entries (row 16h + i, column c) within a block,
// and the buffer size for the padding entries, which the range check turns
// into zeros; the block index goes into the scalar offset.  FP64 blocks are
// the inverses of symmetric Schur complements and are stored as their lower
// triangle, row-major (entry (r, c), r >= c, at r (r + 1) / 2 + c; both
// (r, c) and (c, r) read it): half the bytes of a full block.  FP32 blocks
// are stored whole (nb x nb row-major).
template <typename T>
__host__ __device__ constexpr bool packed_blocks() { return sizeof(T) == 8; }

template <typename T>
__host__ __device__ inline int block_elems(int nb) {
  return packed_blocks<T>() ? nb * (nb + 1) / 2 : nb * nb;
}
template <typename T>
struct BlockSrc {
  __amdgpu_buffer_rsrc_t rs;
  int off[HB];
  int bbytes;
};

template <typename T>
__device__ __forceinline__ BlockSrc<T> block_src(const T* Wg, int nb, int nblk) {
  BlockSrc<T> b;
  // the base and size are wave-uniform: keep them in scalar registers so
  // that the loads need no per-lane resource
  const unsigned long long pa = reinterpret_cast<unsigned long long>(Wg);
  const unsigned plo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)pa);
  const unsigned phi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(pa >> 32));
  T* pu = reinterpret_cast<T*>(((unsigned long long)phi << 32) | plo);
  const int bsz = block_elems<T>(nb);
  const int bytes = __builtin_amdgcn_readfirstlane(nblk * bsz * (int)sizeof(T));
  b.rs = __builtin_amdgcn_make_buffer_rsrc(pu, (short)0, bytes, 0x00020000);
  const int c = threadIdx.x & 31, h = (threadIdx.x >> 5) & 1;
#pragma unroll
  for (int i = 0; i < HB; ++i) {
    const int r = HB * h + i;
    const int hi = r > c ? r : c, lo = r > c ? c : r;
    const int idx = packed_blocks<T>() ? hi * (hi + 1) / 2 + lo : r * nb + c;
    b.off[i] = (r < nb && c < nb) ? idx * (int)sizeof(T) : bytes;
  }
  b.bbytes = __builtin_amdgcn_readfirstlane(bsz * (int)sizeof(T));
  return b;
}

__device__ __forceinline__ void wload_block(const BlockSrc<double>& b, int j, double w[HB]) {
#pragma unroll
  for (int i = 0; i < HB; ++i)
    w[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
        b.rs, b.off[i], __builtin_amdgcn_readfirstlane(j * b.bbytes), 0));
}

__device__ __forceinline__ void wload_block(const BlockSrc<float>& b, int j, float w[HB]) {
#pragma unroll
  for (int i = 0; i < HB; ++i)
    w[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
        b.rs, b.off[i], __builtin_amdgcn_readfirstlane(j * b.bbytes), 0));
}

// dst[e] = *addr(e, fill) for e < n (or `fill` where addr returns nullptr),
// by NT threads with CH loads each in flight before any of them is waited for.
template <int CH, int NT = 64, typename AddrFn>
__device__ __forceinline__ void gather(double* dst, int n, AddrFn addr) {
  const int L = threadIdx.x % NT;
#pragma unroll 1
  for (int e0 = 0; e0 < n; e0 += NT * CH) {
    double v[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = e0 + u * NT + L;
      double fill = 0.0;
      const double* a = (e < n) ? addr(e, fill) : nullptr;
      v[u] = a ? *a : fill;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int e = e0 + u * NT + L;
      if (e < n) dst[e] = v[u];
    }
  }
}

// 1/x from the hardware estimate refined by two Newton steps (x normal).
__device__ __forceinline__ double rcp_d(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Robin coefficients of the face between box cell c (K = kc) and the
// outside cell o (K = ko): beta (paper: alpha H / K_H, or a constant) and
// T^R = |e| / (h / (2 K_c) + beta), with reciprocals in place of divisions.
__device__ __forceinline__ void robin_face(const Geo& g, int a, double kc, double ko, double beta,
                                           double& bt, double& TR) {
  const double Ha = (a == 0 ? g.S[0] : g.S[1]) * g.h;
  bt = g.beta_mode == 1 ? beta : beta * Ha * (kc + ko) * rcp_d(2.0 * kc * ko);
  TR = g.area * 2.0 * kc * rcp_d(g.h + 2.0 * kc * bt);
}

// LDS of the extra permeability tiles of a diagonal tensor with kc entries
// per cell (axes 1.., one halo tile each), placed ahead of a box's other
// arrays; 0 for scalar K.  Even, so that what follows keeps its alignment.
__host__ __device__ inline size_t kx_doubles(int kc, int m0, int m1) {
  return kc > 1 ? ((size_t)(kc - 1) * (m0 + 2) * (m1 + 2) + 1) / 2 * 2 : 0;
}

// The extra tiles at base; returns where the box's own arrays start.
__device__ __forceinline__ double* attach_kx(BoxLds& s, double* base, int kc) {
  s.Kx = base;
  s.ktn = kc > 1 ? (s.m0 + 2) * (s.m1 + 2) : 0;
  return base + kx_doubles(kc, s.m0, s.m1);
}

// After Kt is set: the tile axis 1 reads.
__device__ __forceinline__ void attach_ky(BoxLds& s) { s.Ky = s.ktn ? s.Kx : s.Kt; }

__host__ __device__ inline size_t box_lds_doubles(int m0, int m1, int nrhs, int kc = 1) {
  const int nc = m0 * m1;
  return kx_doubles(kc, m0, m1) + (size_t)(m0 + 2) * (m1 + 2) + 3 * (size_t)nc + (size_t)nrhs * nc +
         (size_t)nrhs * NBW + 2;
}

__device__ __forceinline__ BoxLds carve(double* base, const Box& B, int nrhs, int kc = 1) {
  BoxLds s;
  s.m0 = B.hi[0] - B.lo[0];
  s.m1 = B.hi[1] - B.lo[1];
  const int nc = s.m0 * s.m1;
  base = attach_kx(s, base, kc);
  s.Kt = base;
  attach_ky(s);
  s.Dg = s.Kt + (s.m0 + 2) * (s.m1 + 2);
  s.Tx = s.Dg + nc;
  s.Tn = s.Tx + nc;
  s.X = s.Tn + nc;
  s.Z = align16(base, s.X + (size_t)nrhs * nc);
  return s;
}

// The halo tile of axis a's permeability entries.
__device__ __forceinline__ const double* ktile(const BoxLds& s, int a) { return a == 0 ? s.Kt : s.Ky; }

// K along axis a at global cell (x, y), which must lie in the box or its
// halo.
__device__ __forceinline__ double kat(const BoxLds& s, const Box& B, int x, int y, int a) {
  return ktile(s, a)[(y - B.lo[1] + 1) * (s.m0 + 2) + (x - B.lo[0] + 1)];
}

template <int NT = 64>
__device__ __forceinline__ void coef_box(const Geo& g, const Box& B, double beta, BoxLds& s);

// The tiles of the permeability entries of axes 1.. (diagonal tensor), as
// the Kt tile (LOG: exponentiated here).
template <int NT, bool LOG>
__device__ __forceinline__ void load_kx(const Geo& g, const Box& B, const double* K, const BoxLds& s) {
  if (!s.ktn) return;
  const int W2 = s.m0 + 2, nt = s.ktn;
  gather<1024 / NT, NT>(s.Kx, (g.kc - 1) * nt, [&](int e, double& fill) -> const double* {
    const int a = 1 + e / nt, u = e - (a - 1) * nt;
    const int x = B.lo[0] - 1 + u % W2, y = B.lo[1] - 1 + u / W2;
    fill = LOG ? 0.0 : 1.0;
    return (x >= 0 && x < g.n[0] && !off_domain(g, 1, B.lo[1], y)) ? K + kaxis(g, a) + x + g.n[0] * y
                                                                   : nullptr;
  });
  if (LOG) {
    bsync<NT>();
    for (int e = threadIdx.x % NT; e < (g.kc - 1) * nt; e += NT) s.Kx[e] = exp(s.Kx[e]);
  }
}

// Load the K tile and the matrix coefficients of the box into LDS.
// With LOG, K points to log K and the tile is exponentiated in LDS (cells
// outside the domain read log K = 0, i.e. K = 1, as without).
template <int NT = 64, bool LOG = false>
__device__ __forceinline__ void load_box(const Geo& g, const Box& B, const double* K, double beta, BoxLds& s) {
  const int W2 = s.m0 + 2, H2 = s.m1 + 2;
  gather<1024 / NT, NT>(s.Kt, W2 * H2, [&](int e, double& fill) -> const double* {
    const int x = B.lo[0] - 1 + e % W2, y = B.lo[1] - 1 + e / W2;
    fill = LOG ? 0.0 : 1.0;
    return (x >= 0 && x < g.n[0] && !off_domain(g, 1, B.lo[1], y)) ? K + x + g.n[0] * y : nullptr;
  });
  load_kx<NT, LOG>(g, B, K, s);
  if (LOG) {
    bsync<NT>();
    for (int e = threadIdx.x % NT; e < W2 * H2; e += NT) s.Kt[e] = exp(s.Kt[e]);
  }
  bsync<NT>();
  coef_box<NT>(g, B, beta, s);
}

// Diagonal and couplings of the box matrix from the K tile in LDS.
template <int NT>
__device__ __forceinline__ void coef_box(const Geo& g, const Box& B, double beta, BoxLds& s) {
  const int nc = s.m0 * s.m1;
  const double ih = rcp_d(g.h);
#pragma unroll 1
  for (int loc = threadIdx.x % NT; loc < nc; loc += NT) {
    const int x = B.lo[0] + loc % s.m0, y = B.lo[1] + loc / s.m0;
    double diag = 0.0, tx = 0.0, tn = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double kc = kat(s, B, x, y, a);
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const int ox = x + (a == 0 ? (sd ? 1 : -1) : 0);
        const int oy = y + (a == 1 ? (sd ? 1 : -1) : 0);
        const int t = a == 0 ? ox : oy;
        if (off_domain(g, a, a == 0 ? x : y, t)) {
          if (g.bc_type[2 * a + sd]) diag += 2.0 * kc * g.area * ih;
          continue;
        }
        const double ko = kat(s, B, ox, oy, a);
        const bool inside = ox >= B.lo[0] && ox < B.hi[0] && oy >= B.lo[1] && oy < B.hi[1];
        if (inside) {
          const double T = g.area * 2.0 * kc * ko * rcp_d(kc + ko) * ih;
          diag += T;
          if (sd) {
            if (a == 0) tx = T;
            else tn = T;
          }
        } else {
          double bt, TR;
          robin_face(g, a, kc, ko, beta, bt, TR);
          diag += TR;
        }
      }
    }
    s.Dg[loc] = diag;
    s.Tx[loc] = tx;
    s.Tn[loc] = tn;
  }
  bsync<NT>();
}

// Schur complement of block j (column c, my half) into w: D_j - t W t with
// the coupling t = Tn row tpi to the previously eliminated block, whose
// inverse W w holds on entry (tpi < 0: no previous block, S = D_j).  The
// forward elimination uses tpi = j - 1, the backward one tpi = j.
// Branch-free: every LDS read is unconditional (the addresses stay inside
// the box arrays) and selects pick the tridiagonal entries, so the reads of
// a block issue back to back.
__device__ __forceinline__ void wbuild_t(int nb, int j, int tpi, const BoxLds& s, double w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int cc = c < nb ? c : 0;
  // Unconditional, contiguous reads (paired by the compiler); a missing
  // previous block is a zero factor, not a select on the loads.  Rows past
  // nb read on into the next LDS array of the box and are discarded below.
  const double hpf = tpi >= 0 ? 1.0 : 0.0;
  const double* D = s.Dg + j * nb;
  const double* Tx = s.Tx + j * nb;
  const double* Tp = s.Tn + (tpi >= 0 ? tpi : 0) * nb;
  const double dc = D[cc], txc = Tx[cc];
  const double tc = Tp[cc] * hpf;
  double tr[HB], tpr[HB];
#pragma unroll
  for (int i = 0; i < HB; ++i) {
    tr[i] = Tx[HB * h + i];
    tpr[i] = Tp[HB * h + i];
  }
#pragma unroll
  for (int i = 0; i < HB; ++i) {
    const int r = HB * h + i;
    const int d = r - c;
    double v = d == 0 ? dc : d == -1 ? -tr[i] : d == 1 ? -txc : 0.0;
    v = fma(-tpr[i] * tc, w[i], v);
    w[i] = (r < nb && c < nb) ? v : (d == 0 ? 1.0 : 0.0);
  }
}

// S_j of the forward elimination; w holds W_{j-1} on entry when j > 0.
__device__ __forceinline__ void wbuild(int nb, int j, const BoxLds& s, double w[HB]) {
  wbuild_t(nb, j, j - 1, s, w);
}

// In-place Gauss-Jordan inversion of the block held in w, GJB pivots per
// step (block Gauss-Jordan without pivoting).  For the pivot set K with
// block P = A[K][K], rows R = A[K][:] and columns C = A[:][K], one step
// replaces A[K][j] by P^{-1} A[K][j], A[i][K] by -A[i][K] P^{-1}, A[K][K] by
// P^{-1} and the rest by A - C P^{-1} R: the result of GJB single pivots.
// Lane (c, h) forms v = P^{-1} r with r = A[K][c] (or the unit vector of c
// when c is in K), then updates its 16 rows with the columns C from LDS.
// The owning half writes the pivot rows and the lanes of the pivot columns
// write those columns: one LDS round trip per GJB pivots.  Lines shorter than
// NBW carry identity padding, which a pivot step leaves unchanged.
template <typename T>
__device__ __forceinline__ void wgj_blk(int nb, GjSmem<T>& sm, T w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  bool bad = false;
  for (int k0 = 0; k0 < NBW; k0 += HB) {
    if (k0 >= nb) break;
    const bool own_half = h == (k0 >> 4);
#pragma unroll
    for (int kb = 0; kb < HB; kb += GJB) {
      const int k = k0 + kb;
      if (k >= nb) break;
      T* rb = sm.rowb[(kb / GJB) & 1];
      T* cb = sm.colb[(kb / GJB) & 1];
      const int ck = c - k;
      const bool pc = ck >= 0 && ck < GJB;
      if (own_half) {
#pragma unroll
        for (int m = 0; m < GJB; ++m) rb[GJB * c + m] = w[kb + m];
      }
      if (pc) {
#pragma unroll
        for (int i = 0; i < HB; ++i) cb[ck * NBW + HB * h + i] = w[i];
      }
      wsync();
      T P[GJB][GJB], r[GJB], v[GJB];
#pragma unroll
      for (int j = 0; j < GJB; ++j)
#pragma unroll
        for (int m = 0; m < GJB; ++m) P[m][j] = rb[GJB * (k + j) + m];
      // r = unit vector (pivot-column lanes) or A[K][c], formed arithmetically:
      // a select here becomes a branch per load, each with a full LDS wait
#pragma unroll
      for (int m = 0; m < GJB; ++m)
        r[m] = fma(rb[GJB * c + m], pc ? T(0) : T(1), (pc && ck == m) ? T(1) : T(0));
      const PivBlock<T> q = piv_block(P);
      bad |= !(q.d0 > T(0) && q.da > T(0) && q.s0 > T(0) && q.ds > T(0));
      piv_apply(q, r, v);
#pragma unroll
      for (int i = 0; i < HB; ++i) {
        T acc = pc ? T(0) : w[i];
#pragma unroll
        for (int m = 0; m < GJB; ++m) acc = fma(-cb[m * NBW + HB * h + i], v[m], acc);
        w[i] = acc;
      }
      if (own_half) {
#pragma unroll
        for (int m = 0; m < GJB; ++m) w[kb + m] = v[m];
      }
    }
  }
  if (bad && L == 0) sm.flag |= kFlagNotPD;
  wsync();
}

__device__ __forceinline__ void wgj(int nb, WaveSmem& sm, double w[HB]) { wgj_blk<double>(nb, sm, w); }

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
  if (off_subgrid(g, a, ia, t)) return -1;
  const int stride = (a == 0) ? 1 : g.M[0];
  return sub + (sd ? stride : -stride);
}

// Inner cell of face t on side q of [lo, hi) (2-D).
__device__ __forceinline__ void wgface(const int lo[3], const int hi[3], int q, int t, int& x, int& y) {
  const int a = q >> 1, sd = q & 1;
  const int xe = sd ? hi[0] - 1 : lo[0], ye = sd ? hi[1] - 1 : lo[1];
  x = a == 0 ? xe : lo[0] + t;
  y = a == 0 ? lo[1] + t : ye;
}

__device__ __forceinline__ int bloc(const Box& B, const BoxLds& s, int x, int y) {
  return (x - B.lo[0]) + s.m0 * (y - B.lo[1]);
}

// Physical right-hand side (source, boundary data) of box B into out.
__device__ __forceinline__ void physical_rhs(const Geo& g, const Box& B, const BoxLds& s, const double* f,
                             const double* bcv, double* out) {
  const int nc = s.m0 * s.m1;
  #pragma unroll 1
  for (int loc = lane_id(); loc < nc; loc += 64) {
    const int x = B.lo[0] + loc % s.m0, y = B.lo[1] + loc / s.m0;
    const int ci = x + g.n[0] * y;
    double b = f[ci] * g.vol;
    const int c[3] = {x, y, 0};
    for (int a = 0; a < 2; ++a)
      for (int sd = 0; sd < 2; ++sd) {
        const int t = c[a] + (sd ? 1 : -1);
        if (!off_domain(g, a, c[a], t)) continue;
        const int side = 2 * a + sd;
        const double val = bcv[g.bc_off[side] + bface_index(g, c, a)];
        if (g.bc_type[side]) b += 2.0 * kat(s, B, x, y, a) * g.area / g.h * val;
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
  const double kc = kat(s, B, x, y, a), ko = kat(s, B, ox, oy, a);
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


// ----------------------------------------------------------------- smoothing
// LDS of a smoothing box: the K and p tiles with a one-cell halo, the source,
// the block couplings, the neighbours' Gamma fluxes on the box sides (used
// when the boxes do not overlap) and the boundary data of the box sides on
// the domain boundary, all gathered in one pass; then the matrix
// coefficients, the solution vector and the block staging.
struct SmoothLds {
  BoxLds b;    // Kt, Dg, Tx, Tn, X, Z (Z: 2 x NBW)
  double* P;   // (m0 + 2) x (m1 + 2) pressure tile
  double* F;   // ncell source density
  double* GF;  // 2 (m0 + m1): neighbour flux per face of each box side
  double* BC;  // 2 (m0 + m1): boundary value per face of each box side
};

__host__ __device__ inline size_t smooth_lds_doubles(int m0, int m1, int kc = 1) {
  const size_t nc = (size_t)m0 * m1, nt = (size_t)(m0 + 2) * (m1 + 2);
  return kx_doubles(kc, m0, m1) + 2 * nt + 5 * nc + 4 * (size_t)(m0 + m1) + 4 * NBW + 2;
}

__device__ __forceinline__ int side_off(const BoxLds& s, int q) {
  // faces of side q are numbered along the tangential axis
  return q == 0 ? 0 : q == 1 ? s.m1 : q == 2 ? 2 * s.m1 : 2 * s.m1 + s.m0;
}

// Gather order: [Kt | P | F | Tn | GF | BC] contiguous (after the extra
// permeability tiles of a tensor).
__device__ __forceinline__ SmoothLds carve_smooth(double* base, const Box& B, int kc = 1) {
  SmoothLds r;
  BoxLds& s = r.b;
  s.m0 = B.hi[0] - B.lo[0];
  s.m1 = B.hi[1] - B.lo[1];
  const int nc = s.m0 * s.m1, nt = (s.m0 + 2) * (s.m1 + 2), ns = 2 * (s.m0 + s.m1);
  base = attach_kx(s, base, kc);
  s.Kt = base;
  attach_ky(s);
  r.P = s.Kt + nt;
  r.F = r.P + nt;
  s.Tn = r.F + nc;
  r.GF = s.Tn + nc;
  r.BC = r.GF + ns;
  s.Dg = r.BC + ns;
  s.Tx = s.Dg + nc;
  s.X = s.Tx + nc;
  s.Z = align16(base, s.X + nc);
  return r;
}

// One gather for everything the smoothing solve of box B reads from memory.
// The block couplings come from tcoup (cached by the factorisation) unless
// it is null (then they are left to coef_box).
template <int NT>
__device__ __forceinline__ void stage_smooth(const Geo& g, const Box& B, const SmoothLds& r,
                                             const double* K, const double* p, const double* f,
                                             const double* gflux, const double* bcv,
                                             const double* tcoup) {
  const BoxLds& s = r.b;
  const int m0 = s.m0, m1 = s.m1, W2 = m0 + 2;
  const int nc = m0 * m1, nt = W2 * (m1 + 2), ns = 2 * (m0 + m1);
  const int n0 = g.n[0];
  const int lo0 = B.lo[0], lo1 = B.lo[1];
  const double* tg = tcoup ? tcoup + B.scr : nullptr;
  // per side q: a box side on the domain boundary reads its boundary values;
  // with non-overlapping boxes an interior side reads the neighbour's flux
  const int Mx = g.M[0];
  const int isub = B.sub % Mx, jsub = B.sub / Mx;
  // one gather over the contiguous LDS arrays Kt, P, F, Tn, GF, BC, with
  // about 12 loads per thread in flight (a 24 x 24 box needs one round)
  gather<64 * 48 / NT, NT>(s.Kt, 2 * nt + 2 * nc + 2 * ns, [&](int e, double& fill) -> const double* {
    if (e < 2 * nt) {
      const bool isk = e < nt;
      const int u = isk ? e : e - nt;
      const int y = lo1 - 1 + u / W2, x = lo0 - 1 + (u - (u / W2) * W2);
      fill = isk ? 1.0 : 0.0;
      if (x < 0 || x >= n0 || off_domain(g, 1, lo1, y)) return nullptr;
      return (isk ? K : p) + x + n0 * y;
    }
    e -= 2 * nt;
    if (e < nc) return f + (lo0 + e % m0) + n0 * (lo1 + e / m0);
    e -= nc;
    if (e < nc) return tg ? tg + e : nullptr;
    e -= nc;
    fill = 0.0;
    const bool isgf = e < ns;
    const int u = isgf ? e : e - ns;
    const int q = u < 2 * m1 ? (u < m1 ? 0 : 1) : (u < 2 * m1 + m0 ? 2 : 3);
    const int t = u - (q == 0 ? 0 : q == 1 ? m1 : q == 2 ? 2 * m1 : 2 * m1 + m0);
    const int a = q >> 1, sd = q & 1;
    const int x = a == 0 ? (sd ? B.hi[0] - 1 : lo0) : lo0 + t;
    const int y = a == 1 ? (sd ? B.hi[1] - 1 : lo1) : lo1 + t;
    const int o = (a == 0 ? x : y) + (sd ? 1 : -1);
    const bool dom = off_domain(g, a, a == 0 ? x : y, o);
    if (!isgf) {
      if (!dom) return nullptr;
      const int off = q == 0 ? g.bc_off[0] : q == 1 ? g.bc_off[1] : q == 2 ? g.bc_off[2] : g.bc_off[3];
      const int c3[3] = {x, y, 0};
      return bcv + off + bface_index(g, c3, a);
    }
    if (dom || g.l > 0) return nullptr;
    // neighbour across side q and the face's position on its opposite side
    const int j = B.sub + (a == 0 ? (sd ? 1 : -1) : (sd ? Mx : -Mx));
    const int go = q == 0 ? g.gside_off[1] : q == 1 ? g.gside_off[0] : q == 2 ? g.gside_off[3] : g.gside_off[2];
    const int tj = a == 0 ? y - jsub * g.S[1] : x - isub * g.S[0];
    return gflux + (long long)j * g.gstride + go + tj;
  });
  load_kx<NT, false>(g, B, K, s);
}

// K and p at a cell of the box or its halo.
__device__ __forceinline__ int tile_at(const BoxLds& s, const Box& B, int x, int y) {
  return (y - B.lo[1] + 1) * (s.m0 + 2) + (x - B.lo[0] + 1);
}

// lambda on the face of box cell (x, y) normal to a on side sd of the box,
// from the staged state (Section 3; the neighbour's flux and trace when the
// boxes do not overlap).  bt is the face's beta.
__device__ __forceinline__ double lambda_s(const Geo& g, const Box& B, const SmoothLds& r,
                                           double bt, int x, int y, int a, int sd) {
  const BoxLds& s = r.b;
  const int ox = x + (a == 0 ? (sd ? 1 : -1) : 0), oy = y + (a == 1 ? (sd ? 1 : -1) : 0);
  const int ti = tile_at(s, B, x, y), to = tile_at(s, B, ox, oy);
  const double kc = ktile(s, a)[ti], ko = ktile(s, a)[to];
  if (g.l > 0) {
    // u = K_H (p_c - p_o) / h, pi = p_c - u h / (2 K_c)
    const double u = 2.0 * kc * ko * rcp_d(kc + ko) * (r.P[ti] - r.P[to]) * rcp_d(g.h);
    const double pi = r.P[ti] - u * g.h * 0.5 * rcp_d(kc);
    return -bt * u + pi;
  }
  const int q = 2 * a + sd;
  const double uj = r.GF[side_off(s, q) + (a == 0 ? y - B.lo[1] : x - B.lo[0])];
  const double pij = r.P[to] - uj * g.h * 0.5 * rcp_d(ko);
  return bt * uj + pij;
}

// Right-hand side of the smoothing problem of box B into out (LDS), by NT
// threads: the source on every cell, then the faces of the box sides (x
// sides, then y sides, so that no cell is updated twice at once).
template <int NT>
__device__ __forceinline__ void smooth_rhs(const Geo& g, const Box& B, const SmoothLds& r,
                                           double beta, double* out) {
  const BoxLds& s = r.b;
  const int nc = s.m0 * s.m1;
  const int tid = threadIdx.x % NT;
#pragma unroll 1
  for (int loc = tid; loc < nc; loc += NT) out[loc] = r.F[loc] * g.vol;
  bsync<NT>();
  // both sides of an axis in one pass, except in a box one cell thick
  // along that axis, where they add to the same cells: then one pass each
  auto face = [&](int a, int sd, int t) {
    const int x = a == 0 ? (sd ? B.hi[0] - 1 : B.lo[0]) : B.lo[0] + t;
    const int y = a == 1 ? (sd ? B.hi[1] - 1 : B.lo[1]) : B.lo[1] + t;
    const int c[3] = {x, y, 0};
    const int kind = face_kind(g, B, c, a, sd);
    const double* Ka = ktile(s, a);
    const double kc = Ka[tile_at(s, B, x, y)];
    double add;
    if (kind == kFaceRobin) {
      const int ox = x + (a == 0 ? (sd ? 1 : -1) : 0), oy = y + (a == 1 ? (sd ? 1 : -1) : 0);
      double bt, TR;
      robin_face(g, a, kc, Ka[tile_at(s, B, ox, oy)], beta, bt, TR);
      add = TR * lambda_s(g, B, r, bt, x, y, a, sd);
    } else {
      const double val = r.BC[side_off(s, 2 * a + sd) + t];
      add = kind == kFaceDir ? 2.0 * kc * g.area / g.h * val : -g.area * val;
    }
    out[bloc(B, s, x, y)] += add;
  };
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int nf = a == 0 ? s.m1 : s.m0;
    const int ma = a == 0 ? s.m0 : s.m1;
    if (ma > 1) {
#pragma unroll 1
      for (int u = tid; u < 2 * nf; u += NT) face(a, u >= nf, u - (u >= nf ? nf : 0));
    } else {
#pragma unroll 1
      for (int t = tid; t < nf; t += NT) face(a, 0, t);
      bsync<NT>();
#pragma unroll 1
      for (int t = tid; t < nf; t += NT) face(a, 1, t);
    }
    bsync<NT>();
  }
}

// Smoothing outputs of box B from its solution x (LDS), by NT threads: p on
// Omega_i and Omega_i's own Gamma fluxes (TPFA of the new pressure; the
// Robin formula with the staged lambda when the boxes do not overlap).
template <int NT, typename T>
__device__ __forceinline__ void smooth_out(const Geo& g, const Box& B, const SmoothLds& r, const T* x,
                                           double beta, double* p, double* gflux) {
  const BoxLds& s = r.b;
  const int tid = threadIdx.x % NT;
  int olo[3], ohi[3];
  womega(g, B.sub, olo, ohi);
  const int nfx = g.S[1], nfy = g.S[0];
#pragma unroll 1
  for (int u = tid; u < 2 * (nfx + nfy); u += NT) {
    const int q = u < 2 * nfx ? (u < nfx ? 0 : 1) : (u < 2 * nfx + nfy ? 2 : 3);
    const int t = u - (q == 0 ? 0 : q == 1 ? nfx : q == 2 ? 2 * nfx : 2 * nfx + nfy);
    if (wneighbor(g, B.sub, q) < 0) continue;
    const int a = q >> 1, so = q & 1;
    int cx, cy;
    wgface(olo, ohi, q, t, cx, cy);
    const int ox = cx + (a == 0 ? (so ? 1 : -1) : 0), oy = cy + (a == 1 ? (so ? 1 : -1) : 0);
    const double kc = ktile(s, a)[tile_at(s, B, cx, cy)], ko = ktile(s, a)[tile_at(s, B, ox, oy)];
    const double xc = x[bloc(B, s, cx, cy)];
    double v;
    if (win_box(B, ox, oy)) {
      v = 2.0 * kc * ko * rcp_d(kc + ko) * (xc - x[bloc(B, s, ox, oy)]) * rcp_d(g.h);
    } else {
      double bt, TR;
      robin_face(g, a, kc, ko, beta, bt, TR);
      const double lam = lambda_s(g, B, r, bt, cx, cy, a, so);
      v = TR * (xc - lam) * rcp_d(g.area);
    }
    const int go = q == 0 ? g.gside_off[0] : q == 1 ? g.gside_off[1] : q == 2 ? g.gside_off[2] : g.gside_off[3];
    gflux[(long long)B.sub * g.gstride + go + t] = v;
  }
  const int ncell_o = g.S[0] * g.S[1];
#pragma unroll 1
  for (int t = tid; t < ncell_o; t += NT) {
    const int cx = olo[0] + t % g.S[0], cy = olo[1] + t / g.S[0];
    p[cx + g.n[0] * cy] = x[bloc(B, s, cx, cy)];
  }
}

// ------------------------------------------------------------- block sweeps
// W_j z for the block staged in z (LDS): lane (c, h) sums its 16 rows with
// two accumulators; half_sum completes the column.
__device__ __forceinline__ double wgemv2(const double w[HB], const double* z) {
  const int h = lane_id() >> 5;
  const double2* z2 = reinterpret_cast<const double2*>(z + HB * h);
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int i = 0; i < HB / 2; ++i) {
    const double2 v = z2[i];
    a0 = fma(w[2 * i], v.x, a0);
    a1 = fma(w[2 * i + 1], v.y, a1);
  }
  return half_sum(a0 + a1);
}

// Forward step of block j for all right-hand sides, inverse in w, with jp
// the block eliminated just before j (j - 1 going down the box, j + 1 going
// up; has_prev false for the first block of a chain):
// X_j <- W (X_j + t .* X_jp), t the coupling of j and jp (Tn row min(j, jp)).
// Z: nrhs x NBW doubles of LDS scratch of the calling wave.
__device__ __forceinline__ void fwd_step_d(int nb, int ncell, int j, int jp, bool has_prev,
                                           int nrhs, const BoxLds& s, double* Z,
                                           const double w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int ti = jp < j ? jp : j;
  #pragma unroll 4
  for (int e = L; e < nrhs * NBW; e += 64) {
    const int k = e / NBW, r = e % NBW;
    double v = 0.0;
    if (r < nb) {
      v = s.X[k * ncell + j * nb + r];
      if (has_prev) v += s.Tn[ti * nb + r] * s.X[k * ncell + jp * nb + r];
    }
    Z[k * NBW + r] = v;
  }
  wsync();
  // four right-hand sides at a time: independent product chains overlap
  for (int k0 = 0; k0 < nrhs; k0 += 4) {
    double y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) y[q] = wgemv2(w, Z + min(k0 + q, nrhs - 1) * NBW);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k0 + q < nrhs && h == 0 && c < nb) s.X[(k0 + q) * ncell + j * nb + c] = y[q];
  }
  wsync();
}

__device__ __forceinline__ void fwd_step(int nb, int ncell, int j, int nrhs, const BoxLds& s,
                                         const double w[HB]) {
  fwd_step_d(nb, ncell, j, j - 1, j > 0, nrhs, s, s.Z, w);
}

// Back-substitution step of block j towards block jn (the block solved just
// before it): X_j <- X_j + W (t .* X_jn), t the coupling of j and jn.
__device__ __forceinline__ void bwd_step_d(int nb, int ncell, int j, int jn, int nrhs,
                                           const BoxLds& s, double* Z, const double w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int ti = jn < j ? jn : j;
  #pragma unroll 4
  for (int e = L; e < nrhs * NBW; e += 64) {
    const int k = e / NBW, r = e % NBW;
    Z[k * NBW + r] = (r < nb) ? s.Tn[ti * nb + r] * s.X[k * ncell + jn * nb + r] : 0.0;
  }
  wsync();
  for (int k0 = 0; k0 < nrhs; k0 += 4) {
    double y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) y[q] = wgemv2(w, Z + min(k0 + q, nrhs - 1) * NBW);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k0 + q < nrhs && h == 0 && c < nb) s.X[(k0 + q) * ncell + j * nb + c] += y[q];
  }
  wsync();
}

// Backward step of the one-ended solve: X_j <- X_j + W_j (t_j .* X_{j+1}).
__device__ __forceinline__ void bwd_step(int nb, int ncell, int j, int nrhs, const BoxLds& s,
                                         const double w[HB]) {
  bwd_step_d(nb, ncell, j, j + 1, nrhs, s, s.Z, w);
}

// Meeting block of the two-ended solve, all right-hand sides, Z_m in w:
// X_m <- Z_m (X_m + t_{m-1} .* X_{m-1} + t_m .* X_{m+1}).
__device__ __forceinline__ void mid_step(int nb, int ncell, int m, int nblk, int nrhs,
                                         const BoxLds& s, double* Z, const double w[HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  #pragma unroll 4
  for (int e = L; e < nrhs * NBW; e += 64) {
    const int k = e / NBW, r = e % NBW;
    double v = 0.0;
    if (r < nb) {
      const double* X = s.X + k * ncell;
      v = X[m * nb + r];
      if (m > 0) v = fma(s.Tn[(m - 1) * nb + r], X[(m - 1) * nb + r], v);
      if (m + 1 < nblk) v = fma(s.Tn[m * nb + r], X[(m + 1) * nb + r], v);
    }
    Z[k * NBW + r] = v;
  }
  wsync();
  for (int k0 = 0; k0 < nrhs; k0 += 4) {
    double y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) y[q] = wgemv2(w, Z + min(k0 + q, nrhs - 1) * NBW);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k0 + q < nrhs && h == 0 && c < nb) s.X[(k0 + q) * ncell + m * nb + c] = y[q];
  }
  wsync();
}

// Sweeps with the cached inverses streamed from memory, RING blocks ahead.
__device__ __forceinline__ void forward_cached(const Box& B, const double* Wg, int nrhs, const BoxLds& s) {
  const int nb = B.nb, nblk = B.nblk;
  const long long bs = (long long)nb * nb;
  const BlockSrc<double> src = block_src(Wg, nb, nblk);
  double w[RING][HB];
#pragma unroll
  for (int q = 0; q < RING; ++q)
    if (q < nblk) wload_block(src, q, w[q]);
  for (int j0 = 0; j0 < nblk; j0 += RING) {
#pragma unroll
    for (int q = 0; q < RING; ++q) {
      const int j = j0 + q;
      if (j < nblk) {
        fwd_step(nb, B.ncell, j, nrhs, s, w[q]);
        if (j + RING < nblk) wload_block(src, (j + RING), w[q]);
      }
    }
  }
}

__device__ __forceinline__ void backward_cached(const Box& B, const double* Wg, int nrhs, const BoxLds& s) {
  const int nb = B.nb, nblk = B.nblk;
  const long long bs = (long long)nb * nb;
  const BlockSrc<double> src = block_src(Wg, nb, nblk);
  double w[RING][HB];
  // block j = nblk - 2 - t uses ring slot t % RING
#pragma unroll
  for (int q = 0; q < RING; ++q)
    if (nblk - 2 - q >= 0) wload_block(src, (nblk - 2 - q), w[q]);
  for (int t0 = 0; t0 <= nblk - 2; t0 += RING) {
#pragma unroll
    for (int q = 0; q < RING; ++q) {
      const int j = nblk - 2 - (t0 + q);
      if (j >= 0) {
        bwd_step(nb, B.ncell, j, nrhs, s, w[q]);
        if (j - RING >= 0) wload_block(src, (j - RING), w[q]);
      }
    }
  }
}

// Halves of the two-ended solve of all right-hand sides with cached inverses
// (meeting block m = nblk / 2).  Top: blocks 0 .. m-1 with the forward
// inverses W_j; bottom: blocks nblk-1 .. m+1 with the backward inverses
// W'_j = (D_j - t_j W'_{j+1} t_j)^{-1}.  The forward pass of a half runs
// from its end of the box towards m; the back-substitution from m outwards.
// The inverses stream from memory RING blocks ahead of their use.
__device__ __forceinline__ void twist_fwd_cached(const Box& B, const double* Wg, int nrhs,
                                                 const BoxLds& s, double* Z, bool bottom) {
  const int nb = B.nb, nblk = B.nblk, m = nblk / 2;
  const int cnt = bottom ? nblk - 1 - m : m;
  const int j0 = bottom ? nblk - 1 : 0, dj = bottom ? -1 : 1;
  if (cnt <= 0) return;
  const BlockSrc<double> src = block_src(Wg, nb, nblk);
  double w[RING][HB];
#pragma unroll
  for (int q = 0; q < RING; ++q)
    if (q < cnt) wload_block(src, j0 + dj * q, w[q]);
  for (int t0 = 0; t0 < cnt; t0 += RING) {
#pragma unroll
    for (int q = 0; q < RING; ++q) {
      const int t = t0 + q;
      if (t < cnt) {
        const int j = j0 + dj * t;
        fwd_step_d(nb, B.ncell, j, j - dj, t > 0, nrhs, s, Z, w[q]);
        if (t + RING < cnt) wload_block(src, j0 + dj * (t + RING), w[q]);
      }
    }
  }
}

__device__ __forceinline__ void twist_back_cached(const Box& B, const double* Wg, int nrhs,
                                                  const BoxLds& s, double* Z, bool bottom) {
  const int nb = B.nb, nblk = B.nblk, m = nblk / 2;
  const int cnt = bottom ? nblk - 1 - m : m;
  const int dj = bottom ? 1 : -1;  // direction away from m
  if (cnt <= 0) return;
  const BlockSrc<double> src = block_src(Wg, nb, nblk);
  double w[RING][HB];
#pragma unroll
  for (int q = 0; q < RING; ++q)
    if (q < cnt) wload_block(src, m + dj * (q + 1), w[q]);
  for (int t0 = 0; t0 < cnt; t0 += RING) {
#pragma unroll
    for (int q = 0; q < RING; ++q) {
      const int t = t0 + q;
      if (t < cnt) {
        const int j = m + dj * (t + 1);
        bwd_step_d(nb, B.ncell, j, j - dj, nrhs, s, Z, w[q]);
        if (t + RING < cnt) wload_block(src, m + dj * (t + RING + 1), w[q]);
      }
    }
  }
}

// The whole two-ended solve of all right-hand sides in s.X by one wave:
// Wf holds the forward inverses (blocks < m), Wt the backward inverses
// (blocks > m) and Z_m at block m.
__device__ __forceinline__ void twisted_cached(const Box& B, const double* Wf, const double* Wt,
                                               int nrhs, const BoxLds& s) {
  const int m = B.nblk / 2;
  twist_fwd_cached(B, Wf, nrhs, s, s.Z, false);
  twist_fwd_cached(B, Wt, nrhs, s, s.Z, true);
  double zm[HB];
  wload_block(block_src(Wt, B.nb, B.nblk), m, zm);
  mid_step(B.nb, B.ncell, m, B.nblk, nrhs, s, s.Z, zm);
  twist_back_cached(B, Wf, nrhs, s, s.Z, false);
  twist_back_cached(B, Wt, nrhs, s, s.Z, true);
}

// Forward and backward sweeps of one right-hand side in s.X with the cached
// inverses.  The value of the previous block stays in registers (every lane
// of column c holds it), so a block step is one LDS write of the staged
// vector, the 16-term products and one half-wave exchange.  z points to
// 2 x NBW doubles of LDS (alternating buffers).
__device__ __forceinline__ void sweep1(const Box& B, const double* Wg, const BoxLds& s, double* z) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb, nblk = B.nblk;
  const bool cv = c < nb;
  const long long bs = (long long)nb * nb;
  const BlockSrc<double> src = block_src(Wg, nb, nblk);
  {
    double w[RING][HB];
#pragma unroll
    for (int q = 0; q < RING; ++q)
      if (q < nblk) wload_block(src, q, w[q]);
    double y = 0.0;
    double xn = cv ? s.X[c] : 0.0, tp = 0.0;
    for (int j0 = 0; j0 < nblk; j0 += RING) {
#pragma unroll
      for (int q = 0; q < RING; ++q) {
        const int j = j0 + q;
        if (j < nblk) {
          double* zb = z + (j & 1) * NBW;
          if (h == 0) zb[c] = cv ? fma(tp, y, xn) : 0.0;
          __builtin_amdgcn_wave_barrier();
          const bool more = j + 1 < nblk;
          xn = (more && cv) ? s.X[(j + 1) * nb + c] : 0.0;
          tp = (more && cv) ? s.Tn[j * nb + c] : 0.0;
          y = wgemv2(w[q], zb);
          if (h == 0 && cv) s.X[j * nb + c] = y;
          if (j + RING < nblk) wload_block(src, (j + RING), w[q]);
        }
      }
    }
  }
  {
    double w[RING][HB];
#pragma unroll
    for (int q = 0; q < RING; ++q)
      if (nblk - 2 - q >= 0) wload_block(src, (nblk - 2 - q), w[q]);
    // x_{nblk-1} = w_{nblk-1} is final; every lane of column c reads it
    __builtin_amdgcn_wave_barrier();
    double xnext = cv ? s.X[(nblk - 1) * nb + c] : 0.0;
    double tj = (nblk >= 2 && cv) ? s.Tn[(nblk - 2) * nb + c] : 0.0;
    double wj = (nblk >= 2 && cv) ? s.X[(nblk - 2) * nb + c] : 0.0;
    for (int t0 = 0; t0 <= nblk - 2; t0 += RING) {
#pragma unroll
      for (int q = 0; q < RING; ++q) {
        const int j = nblk - 2 - (t0 + q);
        if (j >= 0) {
          double* zb = z + (j & 1) * NBW;
          if (h == 0) zb[c] = cv ? tj * xnext : 0.0;
          __builtin_amdgcn_wave_barrier();
          const double wcur = wj;
          tj = (j >= 1 && cv) ? s.Tn[(j - 1) * nb + c] : 0.0;
          wj = (j >= 1 && cv) ? s.X[(j - 1) * nb + c] : 0.0;
          xnext = wcur + wgemv2(w[q], zb);
          if (h == 0 && cv) s.X[j * nb + c] = xnext;
          if (j - RING >= 0) wload_block(src, (j - RING), w[q]);
        }
      }
    }
  }
  wsync();
}

// ---------------------------------------------------------- twisted sweep
// The block-tridiagonal box system solved from both ends towards the
// meeting block m = nblk / 2 (a twisted block factorisation):
//   top:     z_j = W_j (b_j + t_{j-1} z_{j-1}),    j = 0 .. m-1
//   bottom:  z_j = W'_j (b_j + t_j z_{j+1}),       j = nblk-1 .. m+1
//   meet:    x_m = Z_m (b_m + t_{m-1} z_{m-1} + t_m z_{m+1})
//   top:     x_j = z_j + W_j (t_j x_{j+1}),        j = m-1 .. 0
//   bottom:  x_j = z_j + W'_j (t_{j-1} x_{j-1}),   j = m+1 .. nblk-1
// with the forward inverses W_j, the backward inverses W'_j =
// (D_j - t_j W'_{j+1} t_j)^{-1} and Z_m = (S_m - t_m W'_{m+1} t_m)^{-1}, S_m
// the forward Schur complement of block m.  All of them are symmetric, so
// the column-per-lane products of sweep1 apply.  The two halves touch
// disjoint blocks of s.X and may run on two waves at once; each half needs
// its own 2 x NBW doubles of LDS staging z.

// One half of the twisted sweep: block j = j0 + dj * b for the b-th block
// away from the end (b = 0 .. cnt-1).  The register ring holds block b in
// slot (b + o) % RING, with o chosen so that the last block of the forward
// pass sits in slot RING-1: the back pass then finds its first RING blocks
// in place (slot RING-1-q for its q-th block) and the slot of every block
// stays a compile-time index.
struct TwistHalf {
  BlockSrc<double> src;
  int cnt, j0, dj, o;
};

__device__ __forceinline__ TwistHalf twist_half(const Box& B, const double* Wg, int m, bool bottom) {
  TwistHalf hf;
  hf.src = block_src(Wg, B.nb, B.nblk);
  hf.cnt = bottom ? B.nblk - 1 - m : m;
  hf.j0 = bottom ? B.nblk - 1 : 0;
  hf.dj = bottom ? -1 : 1;
  hf.o = hf.cnt > 0 ? (RING - hf.cnt % RING) % RING : 0;
  return hf;
}

// First RING blocks of the forward pass into the ring (block b in slot
// (b + o) % RING).
__device__ __forceinline__ void twist_preload(const TwistHalf& hf, double w[RING][HB]) {
#pragma unroll
  for (int q = 0; q < RING; ++q) {
    const int b = (q - hf.o + RING) % RING;
    if (b < hf.cnt) wload_block(hf.src, hf.j0 + hf.dj * b, w[q]);
  }
}

// Forward half (ring preloaded); z_j replaces b_j in s.X.
__device__ __forceinline__ void twist_fwd(const Box& B, const TwistHalf& hf, const BoxLds& s,
                                          double* z, bool bottom, double w[RING][HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb;
  const bool cv = c < nb;
  const int cnt = hf.cnt;
  if (cnt <= 0) return;
  double y = 0.0, tp = 0.0;
  double xn = cv ? s.X[hf.j0 * nb + c] : 0.0;
  for (int v0 = 0; v0 < cnt + hf.o; v0 += RING) {
#pragma unroll
    for (int q = 0; q < RING; ++q) {
      const int t = v0 + q - hf.o;
      if (t >= 0 && t < cnt) {
        const int j = hf.j0 + hf.dj * t;
        double* zb = z + (t & 1) * NBW;
        if (h == 0) zb[c] = cv ? fma(tp, y, xn) : 0.0;
        __builtin_amdgcn_wave_barrier();
        const bool more = t + 1 < cnt;
        const int jn = j + hf.dj;             // next block of this half
        const int ti = bottom ? jn : j;       // coupling between j and jn
        xn = (more && cv) ? s.X[jn * nb + c] : 0.0;
        tp = (more && cv) ? s.Tn[ti * nb + c] : 0.0;
        y = wgemv2(w[q], zb);
        if (h == 0 && cv) s.X[j * nb + c] = y;
        if (t + RING < cnt) wload_block(hf.src, hf.j0 + hf.dj * (t + RING), w[q]);
      }
    }
  }
}

// Meeting block: x_m from b_m and the neighbouring z of both halves; zm
// holds Z_m in the block register layout.
__device__ __forceinline__ void twist_mid(const Box& B, const double zm[HB], const BoxLds& s,
                                          double* z, int m) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb, nblk = B.nblk;
  const bool cv = c < nb;
  double v = 0.0;
  if (cv) {
    v = s.X[m * nb + c];
    if (m > 0) v = fma(s.Tn[(m - 1) * nb + c], s.X[(m - 1) * nb + c], v);
    if (m + 1 < nblk) v = fma(s.Tn[m * nb + c], s.X[(m + 1) * nb + c], v);
  }
  if (h == 0) z[c] = v;
  __builtin_amdgcn_wave_barrier();
  const double y = wgemv2(zm, z);
  if (h == 0 && cv) s.X[m * nb + c] = y;
}

// Back-substitution half, outwards from the meeting block.  With
// have_ring the ring is the one the forward pass of this half left behind.
__device__ __forceinline__ void twist_back(const Box& B, const TwistHalf& hf, const BoxLds& s,
                                           double* z, int m, bool bottom, bool have_ring,
                                           double w[RING][HB]) {
  const int L = lane_id();
  const int c = L & 31, h = L >> 5;
  const int nb = B.nb;
  const bool cv = c < nb;
  const int cnt = hf.cnt;
  if (cnt <= 0) return;
  if (!have_ring) {
#pragma unroll
    for (int q = 0; q < RING; ++q) {
      const int b = cnt - 1 - q;
      if (b >= 0) wload_block(hf.src, hf.j0 + hf.dj * b, w[RING - 1 - q]);
    }
  }
  const int jf = hf.j0 + hf.dj * (cnt - 1);  // first block of the back pass (next to m)
  double xnext = cv ? s.X[m * nb + c] : 0.0;
  double tj = cv ? s.Tn[(bottom ? jf - 1 : jf) * nb + c] : 0.0;
  double wj = cv ? s.X[jf * nb + c] : 0.0;
  for (int v0 = 0; v0 < cnt; v0 += RING) {
#pragma unroll
    for (int q = 0; q < RING; ++q) {
      const int t = v0 + q;
      if (t < cnt) {
        const int b = cnt - 1 - t;
        const int j = hf.j0 + hf.dj * b;
        double* zb = z + (t & 1) * NBW;
        if (h == 0) zb[c] = cv ? tj * xnext : 0.0;
        __builtin_amdgcn_wave_barrier();
        const double wcur = wj;
        const bool more = t + 1 < cnt;
        const int jn = j - hf.dj;             // next block, away from m
        tj = (more && cv) ? s.Tn[(bottom ? jn - 1 : jn) * nb + c] : 0.0;
        wj = (more && cv) ? s.X[jn * nb + c] : 0.0;
        xnext = wcur + wgemv2(w[RING - 1 - q], zb);
        if (h == 0 && cv) s.X[j * nb + c] = xnext;
        if (b - RING >= 0) wload_block(hf.src, hf.j0 + hf.dj * (b - RING), w[RING - 1 - q]);
      }
    }
  }
}

// The whole twisted sweep of one right-hand side by the NT threads of a
// box.  With NT >= 128 the two halves run on waves 0 and 1 at once, each
// keeping its ring from the forward into the back pass; the caller has
// preloaded the ring of its half (twist_preload) and wave 0 the meeting
// block (zm), before staging, so that their memory latency is hidden.  With
// NT = 64 one wave runs the halves one after the other and loads as it
// goes.  The arithmetic is the same in both cases, and so is the result.
// Wf: forward inverses, Wt: backward inverses and Z_m; z: 4 x NBW doubles.
template <int NT>
__device__ __forceinline__ void sweep_twisted(const Box& B, const double* Wf, const double* Wt,
                                              const BoxLds& s, double* z, double w[RING][HB],
                                              const double zm[HB]) {
  const int wv = threadIdx.x >> 6;
  const int m = B.nblk / 2;
  double* za = z;
  double* zb = z + 2 * NBW;
  const TwistHalf top = twist_half(B, Wf, m, false);
  const TwistHalf bot = twist_half(B, Wt, m, true);
  if (NT == 64) {
    twist_preload(top, w);
    twist_fwd(B, top, s, za, false, w);
    twist_preload(bot, w);
    twist_fwd(B, bot, s, zb, true, w);
  } else if (wv == 0) {
    twist_fwd(B, top, s, za, false, w);
  } else if (wv == 1) {
    twist_fwd(B, bot, s, zb, true, w);
  }
  bsync<NT>();
  if (wv == 0) twist_mid(B, zm, s, za, m);
  bsync<NT>();
  if (NT == 64) {
    twist_back(B, top, s, za, m, false, false, w);
    twist_back(B, bot, s, zb, m, true, false, w);
  } else if (wv == 0) {
    twist_back(B, top, s, za, m, false, true, w);
  } else if (wv == 1) {
    twist_back(B, bot, s, zb, m, true, true, w);
  }
  bsync<NT>();
}

}  // namespace wave
}  // namespace mrcm
