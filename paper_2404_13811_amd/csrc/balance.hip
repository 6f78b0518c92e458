// Conservation and continuity measures of a solution state (Section 5's
// error measures; the discrete statements behind them are the cell mass
// balance of the mixed system and the interface equations int_ujump and
// int_pjump):
//
//   cell residual    r_c = sum_faces |e| u_e - f_c h^d   (u the output
//                    velocities: skeleton faces carry the owner's flux)
//   boundary outflow Q_q = sum over the faces of domain side q of |e| u.n
//   flux jump        sum_e |e| mu (u_i + u_j)   per interface Gamma_ij and
//                    test function mu (u_i, u_j: each side's own outward
//                    flux), relative to sum_e |e| |mu| (|u_i| + |u_j|)
//   pressure jump    sum_e |e| mu (pi_i - pi_j), pi = p_c - u h / (2 K_c),
//                    relative to sum_e |e| |mu| (|pi_i| + |pi_j|)
//
// Right after the MRCM-O assembly the two jumps are the residual of the
// interface system row by row (the state holds pbar + sum X P and
// ubar + sum X u), which is how the interface solve is checked.  Sums are
// deterministic: fixed per-workgroup trees, partials combined in a fixed
// order; maxima go through integer atomics on the bit patterns of
// non-negative doubles, whose order is the order of the values.
#include "local_common.h"

#include <mutex>

namespace mrcm {
namespace {

constexpr int RB = 256;

__device__ __forceinline__ void iface_box(const Geo& g, int sub, int lo[3], int hi[3]) {
  int r = sub;
  for (int a = 0; a < 3; ++a) {
    const int Ma = (a < g.d) ? g.M[a] : 1;
    const int ia = r % Ma;
    r /= Ma;
    lo[a] = (a < g.d) ? ia * g.S[a] : 0;
    hi[a] = (a < g.d) ? lo[a] + g.S[a] : 1;
  }
}

__device__ __forceinline__ void side_cell(const int lo[3], const int hi[3], int q, int t, int c[3]) {
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

__device__ __forceinline__ unsigned long long dbits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}

// Fixed-order sum of one value per thread of a 256-thread workgroup.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = RB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = RB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Per cell: mass-balance residual (to res when not null); per workgroup:
// max |r_c|, max sum |e||u_e|, sum f_c h^d and the outflow of every domain
// side, into partial[b * kBalParts + k].
__global__ void __launch_bounds__(RB) k_cell_balance(Geo g, const double* __restrict__ K,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ gflux,
                                                     const double* __restrict__ bcv,
                                                     const double* __restrict__ f,
                                                     double* __restrict__ res,
                                                     double* __restrict__ partial) {
  __shared__ double sh[RB];
  const int ci = blockIdx.x * RB + threadIdx.x;
  double r = 0.0, ab = 0.0, src = 0.0, out[6] = {0, 0, 0, 0, 0, 0};
  if (ci < g.ncells) {
    int c[3], own[3];
    const int sub = cell_owner(g, ci, c, own);
    double sum = 0.0;
    for (int a = 0; a < g.d; ++a)
      for (int s = 0; s < 2; ++s) {
        const double u = state_face_u(g, K, p, gflux, bcv, c, ci, own, sub, a, s);
        sum += g.area * u;
        ab += g.area * fabs(u);
        const int o = c[a] + (s ? 1 : -1);
        if (off_domain(g, a, c[a], o)) out[2 * a + s] = g.area * u;
      }
    src = f[ci] * g.vol;
    r = sum - src;
    if (res) res[ci] = r;
  }
  double* P = partial + (long long)blockIdx.x * kBalParts;
  const double m0 = block_max(fabs(r), sh);
  const double m1 = block_max(ab, sh);
  const double s0 = block_sum(src, sh);
  double o[6];
  for (int q = 0; q < 6; ++q) o[q] = block_sum(out[q], sh);
  if (threadIdx.x == 0) {
    P[0] = m0;
    P[1] = m1;
    P[2] = s0;
    for (int q = 0; q < 6; ++q) P[3 + q] = o[q];
  }
}

// Partials combined in workgroup order (one thread per quantity).
__global__ void k_cell_balance_final(const double* __restrict__ partial, int nb,
                                     double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k >= kBalParts) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double v = partial[(long long)b * kBalParts + k];
    acc = k < 2 ? fmax(acc, v) : acc + v;
  }
  out[k] = acc;
}

// One wave per interface: for each of its 2 p equation rows the moment of
// the jump (to mom[row] when not null) and a moment of magnitudes; the
// largest ratio over the flux rows and over the pressure rows goes to
// jmax[0] and jmax[1] (atomic max on the bits).  A ratio above tol raises
// kFlagSingular (tol <= 0: no check).  The magnitudes are those of the two
// sides' values (|u_i| + |u_j|, |pi_i| + |pi_j|), or, with the interface
// traces given (tr.X not null), those of every term of the interface
// equation, sum_k |X_i^k| |u_i^k| + |ubar_i| + (the same for j): the ratio
// is then the row's componentwise backward error |G X - r| / (|G||X| + |r|)
// of the interface solve, which cancellation in an ill-conditioned system
// does not inflate.
// The measures of one interface by one wave; the row maxima are returned
// to lane 0's worst[].
__device__ __forceinline__ void jumps_one(const Geo& g, const Iface F, const Seed* __restrict__ basis,
                                          const double* __restrict__ K, const double* __restrict__ p,
                                          const double* __restrict__ gflux, double* __restrict__ mom,
                                          const JumpTerms& tr, double worst[2]) {
  const int L = threadIdx.x & 63;
  const int qi = 2 * F.axis + 1, qj = 2 * F.axis;
  K += kaxis(g, F.axis);  // the entry normal to the interface
  int ilo[3], ihi[3], jlo[3], jhi[3];
  iface_box(g, F.i, ilo, ihi);
  iface_box(g, F.j, jlo, jhi);
  int nf = 1;
  for (int b = 0; b < g.d; ++b)
    if (b != F.axis) nf *= g.S[b];
  const long long bi = (long long)F.i * g.gstride + g.gside_off[qi];
  const long long bj = (long long)F.j * g.gstride + g.gside_off[qj];
  // lanes in NG groups of nf faces when the faces of a side divide the wave:
  // group q takes the seeds q, q + NG, ... of the two sides (all loads of a
  // lane independent), group 0 also the jump itself and the particular
  // solution's terms; otherwise one group strides over the faces
  const int NG = (nf <= 64 && 64 % nf == 0) ? 64 / nf : 1;
  const int grp = NG > 1 ? L / nf : 0;
  const int tl = NG > 1 ? L % nf : L;
  const int tstep = NG > 1 ? nf : 64;
  const int ni = tr.X ? tr.seed_off[F.i + 1] - tr.seed_off[F.i] : 0;
  const int nseed = tr.X ? ni + tr.seed_off[F.j + 1] - tr.seed_off[F.j] : 0;
  for (int rr = 0; rr < 2 * F.nbasis; ++rr) {
    const int kind = rr / F.nbasis;  // 0 flux, 1 pressure
    const Seed mu = basis[F.basis0 + rr % F.nbasis];
    double m = 0.0, sc = 0.0;
    for (int t = tl; t < nf; t += tstep) {
      int ci[3];
      side_cell(ilo, ihi, qi, t, ci);
      const double w = g.area * seed_value(g, mu, ilo, ihi, ci);
      double a = 0.0, b = 0.0;
      if (grp == 0) {
        const double ui = gflux[bi + t], uj = gflux[bj + t];
        if (kind == 0) {
          a = ui;
          b = uj;
          m += w * (a + b);
        } else {
          int cj[3];
          side_cell(jlo, jhi, qj, t, cj);
          const int ii = gcell(g, ci), jj = gcell(g, cj);
          a = p[ii] - ui * g.h / (2.0 * K[ii]);
          b = p[jj] - uj * g.h / (2.0 * K[jj]);
          m += w * (a - b);
        }
      }
      if (tr.X) {
        // every term of the row: the seeds' traces times |X|, the particular
        // solution's trace
        double mag = 0.0;
        if (grp == 0)
          mag = fabs(kind == 0 ? tr.ubar[bi + t] : tr.pibar[bi + t]) +
                fabs(kind == 0 ? tr.ubar[bj + t] : tr.pibar[bj + t]);
        for (int e = grp; e < nseed; e += NG) {
          const int side = e >= ni;
          const int sub = side ? F.j : F.i;
          const int k = tr.seed_off[sub] + (side ? e - ni : e);
          const long long so = (side ? g.gside_off[qj] : g.gside_off[qi]) + t;
          const long long ek = (long long)k * g.gstride + so;
          const double v = kind == 0 ? tr.tr_u[ek]
                                     : tr.tr_beta[(long long)sub * g.gstride + so] * tr.tr_u[ek] +
                                           tr.tr_phi[ek];
          mag += fabs(tr.X[k] * v);
        }
        sc += fabs(w) * mag;
      } else if (grp == 0) {
        sc += fabs(w) * (fabs(a) + fabs(b));
      }
    }
    // fixed-order wave sums
    for (int off = 32; off > 0; off >>= 1) {
      m += __shfl_xor(m, off);
      sc += __shfl_xor(sc, off);
    }
    if (mom && L == 0) mom[F.row0 + rr] = m;
    // 0 / 0 (a row with no terms at all) is a satisfied row
    const double ratio = sc > 0.0 ? fabs(m) / sc : (m == 0.0 ? 0.0 : INFINITY);
    // a NaN ratio counts as the worst
    worst[kind] = (ratio == ratio) ? fmax(worst[kind], ratio) : INFINITY;
  }
}

// Four waves per workgroup, each taking interfaces in a grid-stride loop;
// the workgroup's maxima go out with one atomic pair (atomics of every
// interface on the same two words serialise in L2).
__global__ void __launch_bounds__(256) k_jumps(Geo g, const Iface* __restrict__ ifc, int nifc,
                                               const Seed* __restrict__ basis,
                                               const double* __restrict__ K,
                                               const double* __restrict__ p,
                                               const double* __restrict__ gflux,
                                               double* __restrict__ mom,
                                               unsigned long long* __restrict__ jmax, double tol,
                                               int* flags, JumpTerms tr) {
  __shared__ double wmax[4][2];
  const int wv = threadIdx.x >> 6;
  double worst[2] = {0.0, 0.0};
  for (int f = blockIdx.x * 4 + wv; f < nifc; f += gridDim.x * 4)
    jumps_one(g, ifc[f], basis, K, p, gflux, mom, tr, worst);
  if ((threadIdx.x & 63) == 0) {
    wmax[wv][0] = worst[0];
    wmax[wv][1] = worst[1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double w0 = 0.0, w1 = 0.0;
    for (int u = 0; u < 4; ++u) {
      // a NaN or infinite ratio wins
      w0 = (wmax[u][0] == wmax[u][0]) ? fmax(w0, wmax[u][0]) : INFINITY;
      w1 = (wmax[u][1] == wmax[u][1]) ? fmax(w1, wmax[u][1]) : INFINITY;
    }
    atomicMax(&jmax[0], dbits(w0));
    atomicMax(&jmax[1], dbits(w1));
    if (tol > 0.0 && !(fmax(w0, w1) <= tol)) atomicOr(flags, kFlagSingular);
  }
}

// Partial sums of (a - b)^2 and b^2 over a fixed grid-stride partition.
__global__ void __launch_bounds__(RB) k_sq_dist(const double* __restrict__ a,
                                                const double* __restrict__ b, long long n,
                                                double* __restrict__ partial) {
  __shared__ double sh[RB];
  double d2 = 0.0, b2 = 0.0;
  for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < n; i += (long long)gridDim.x * RB) {
    const double d = a[i] - b[i];
    d2 += d * d;
    b2 += b[i] * b[i];
  }
  const double s0 = block_sum(d2, sh);
  const double s1 = block_sum(b2, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s0;
    partial[2 * blockIdx.x + 1] = s1;
  }
}

__global__ void k_sq_dist_final(const double* __restrict__ partial, int nb, double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k >= 2) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) acc += partial[2 * b + k];
  out[k] = acc;
}

}  // namespace

hipError_t launch_sq_dist(const double* a, const double* b, long long n, double* partial,
                          double* out, hipStream_t s) {
  const int nb = 256;
  hipLaunchKernelGGL(k_sq_dist, dim3(nb), dim3(RB), 0, s, a, b, n, partial);
  hipLaunchKernelGGL(k_sq_dist_final, dim3(1), dim3(64), 0, s, partial, nb, out);
  return hipGetLastError();
}

// Scratch of mrcm_get_balance_static: a file-scope device array (one copy
// per GPU, held until the process ends), so that the call allocates
// nothing.  Host code never passes the array's name to a kernel: it uses the
// device address hipGetSymbolAddress returns, kept per device.
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
std::mutex scratch_mu;
double* scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(double** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    double* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = p;
  }
  *ptr = scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_cell_balance(const Geo& g, const double* K, const double* p, const double* gflux,
                               const double* bcv, const double* f, double* res, double* partial,
                               int max_blocks, double* out, hipStream_t s) {
  const int nb = (g.ncells + RB - 1) / RB;
  if (nb > max_blocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cell_balance, dim3(nb), dim3(RB), 0, s, g, K, p, gflux, bcv, f, res, partial);
  hipLaunchKernelGGL(k_cell_balance_final, dim3(1), dim3(64), 0, s, partial, nb, out);
  return hipGetLastError();
}

int cell_balance_blocks(const Geo& g) { return (g.ncells + RB - 1) / RB; }

hipError_t launch_jumps(const Geo& g, const Iface* ifc, int nifc, const Seed* basis, const double* K,
                        const double* p, const double* gflux, double* mom,
                        unsigned long long* jmax, double tol, int* flags, hipStream_t s,
                        const JumpTerms* terms) {
  if (nifc <= 0) return hipSuccess;
  JumpTerms tr{};
  if (terms) tr = *terms;
  const int nblk = std::min((nifc + 3) / 4, 2048);
  hipLaunchKernelGGL(k_jumps, dim3(nblk), dim3(256), 0, s, g, ifc, nifc, basis, K, p, gflux, mom, jmax,
                     tol, flags, tr);
  return hipGetLastError();
}

}  // namespace mrcm
