// Local problems of MRCM-OS on gfx950: batched block-tridiagonal LDL^T
// factorisations with explicit block inverses, multi-RHS solves, the seed
// (basis-function) solves with interface-trace extraction, the particular
// problems, and the colored smoothing sweep.
//
// Algorithm 1 of the paper factors each local matrix once and reuses it for
// every right-hand side (Steps 1-2, 6-7).  Here each local matrix, ordered
// x fastest, is block tridiagonal with dense diagonal blocks D_j (one line or
// plane of cells) and diagonal couplings C_j = -diag(t_j).  Its block LDL^T
// factor is stored as the inverses W_j = S_j^{-1} of the Schur complements
//   S_0 = D_0,  S_j = D_j - diag(t_{j-1}) W_{j-1} diag(t_{j-1}),
// so that a solve is a chain of dense block products:
//   forward   w_j = W_j (b_j + t_{j-1} .* w_{j-1})
//   backward  x_j = w_j + W_j (t_j .* x_{j+1}).
// One workgroup owns one box; the block being inverted lives in LDS.
#include "local_common.h"

namespace mrcm {

namespace {

constexpr int NT = kLocalThreads;
constexpr int LDW = kMaxBlock + 1;  // padded LDS row stride of a block

struct LocalSmem {
  double W[kMaxBlock * LDW];       // block being built / inverted
  double Z[kMaxRhs * kMaxBlock];   // right-hand sides of one block
  double diag[kMaxBlock];
  double tprev[kMaxBlock];
  double tnext[kMaxBlock];
  double tx[kMaxBlock];
  double ty[kMaxBlock];
  double red[NT / 64];
  int flag;
};

__device__ __forceinline__ void block_cell(const Box& B, int d, int j, int a, int c[3]) {
  const int m0 = B.hi[0] - B.lo[0];
  c[0] = B.lo[0] + a % m0;
  if (d == 2) {
    c[1] = B.lo[1] + j;
    c[2] = 0;
  } else {
    c[1] = B.lo[1] + a / m0;
    c[2] = B.lo[2] + j;
  }
}

// Coefficients of block j into LDS (diag, in-block couplings, coupling to
// block j+1 in tnext).  tprev must already hold the coupling to block j-1.
__device__ void load_block_coefs(const Geo& g, const Box& B, const double* K, double beta, int j,
                                 LocalSmem& sm) {
  for (int a = threadIdx.x; a < B.nb; a += NT) {
    int c[3];
    block_cell(B, g.d, j, a, c);
    CellCoef cc = cell_coef(g, B, K, c, beta);
    sm.diag[a] = cc.diag;
    sm.tx[a] = cc.tp[0];
    sm.ty[a] = (g.d == 3) ? cc.tp[1] : 0.0;
    sm.tnext[a] = cc.tp[g.d - 1];
  }
}

// S_j = D_j - diag(tprev) W_{j-1} diag(tprev), in place over W_{j-1}.
__device__ void build_schur(const Box& B, int d, LocalSmem& sm, bool first) {
  const int nb = B.nb;
  const int m0 = B.hi[0] - B.lo[0];
  for (int e = threadIdx.x; e < nb * nb; e += NT) {
    const int r = e / nb, c = e % nb;
    double v = 0.0;
    if (r == c) {
      v = sm.diag[r];
    } else if (c == r + 1 && (r % m0) < m0 - 1) {
      v = -sm.tx[r];
    } else if (r == c + 1 && (c % m0) < m0 - 1) {
      v = -sm.tx[c];
    } else if (d == 3 && c == r + m0) {
      v = -sm.ty[r];
    } else if (d == 3 && r == c + m0) {
      v = -sm.ty[c];
    }
    if (!first) v -= sm.tprev[r] * sm.tprev[c] * sm.W[r * LDW + c];
    sm.W[r * LDW + c] = v;
  }
}

// In-place Gauss-Jordan inversion of the SPD block in LDS (no pivoting: the
// pivots are Schur-complement diagonals, positive for an SPD matrix).
__device__ void gj_invert(int nb, LocalSmem& sm) {
  constexpr int EPT = (kMaxBlock * kMaxBlock + NT - 1) / NT;
  for (int k = 0; k < nb; ++k) {
    __syncthreads();
    const double piv = sm.W[k * LDW + k];
    if (!(piv > 0.0) && threadIdx.x == 0) sm.flag |= kFlagNotPD;
    const double ip = 1.0 / piv;
    double wak[EPT], wkb[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = threadIdx.x + q * NT;
      if (e < nb * nb) {
        const int r = e / nb, c = e % nb;
        wak[q] = sm.W[r * LDW + k];
        wkb[q] = sm.W[k * LDW + c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = threadIdx.x + q * NT;
      if (e < nb * nb) {
        const int r = e / nb, c = e % nb;
        double v;
        if (r == k && c == k) v = ip;
        else if (r == k) v = wkb[q] * ip;
        else if (c == k) v = -wak[q] * ip;
        else v = sm.W[r * LDW + c] - wak[q] * wkb[q] * ip;
        sm.W[r * LDW + c] = v;
      }
    }
  }
  __syncthreads();
}

// y[k][r] = sum_c W[r][c] z[k][c] for k < nrhs; W row-major with stride ldw,
// z in LDS (stride kMaxBlock), result to global y (stride ystride).
template <typename WT>
__device__ void block_gemv(int nb, int nrhs, const WT* W, int ldw, const double* z, double* y,
                           long long ystride, const double* add) {
  for (int o = threadIdx.x; o < nb * nrhs; o += NT) {
    const int k = o / nb, r = o % nb;
    double acc = 0.0;
    for (int c = 0; c < nb; ++c) acc += (double)W[c * ldw + r] * z[k * kMaxBlock + c];
    if (add) acc += add[k * ystride + r];
    y[k * ystride + r] = acc;
  }
}

// Forward+backward sweeps with cached inverses (global), right-hand sides
// and results in scr[k * ncell + cell].  If `fused_first` the inverse of
// block 0..nblk-1 is NOT used for the forward sweep (already done).
__device__ void backward_sweep(const Geo& g, const Box& B, const double* K, double beta,
                               const double* Wg, double* scr, int nrhs, LocalSmem& sm) {
  const int nb = B.nb;
  for (int j = B.nblk - 2; j >= 0; --j) {
    __syncthreads();
    load_block_coefs(g, B, K, beta, j, sm);
    __syncthreads();
    for (int o = threadIdx.x; o < nb * nrhs; o += NT) {
      const int k = o / nb, r = o % nb;
      sm.Z[k * kMaxBlock + r] = sm.tnext[r] * scr[(long long)k * B.ncell + (j + 1) * nb + r];
    }
    __syncthreads();
    const double* Wj = Wg + (long long)j * nb * nb;
    for (int o = threadIdx.x; o < nb * nrhs; o += NT) {
      const int k = o / nb, r = o % nb;
      double acc = 0.0;
      for (int c = 0; c < nb; ++c) acc += Wj[c * nb + r] * sm.Z[k * kMaxBlock + c];
      scr[(long long)k * B.ncell + j * nb + r] += acc;
    }
  }
  __syncthreads();
}

// Factor the box and run the forward sweep on nrhs right-hand sides already
// in scr (overwritten by w).  Inverses go to Wg.
__device__ void factor_forward(const Geo& g, const Box& B, const double* K, double beta,
                               double* Wg, double* scr, int nrhs, LocalSmem& sm) {
  const int nb = B.nb;
  for (int j = 0; j < B.nblk; ++j) {
    __syncthreads();
    // coupling to the previous block becomes tprev
    if (j > 0)
      for (int a = threadIdx.x; a < nb; a += NT) sm.tprev[a] = sm.tnext[a];
    __syncthreads();
    load_block_coefs(g, B, K, beta, j, sm);
    __syncthreads();
    build_schur(B, g.d, sm, j == 0);
    gj_invert(nb, sm);
    double* Wj = Wg + (long long)j * nb * nb;
    for (int e = threadIdx.x; e < nb * nb; e += NT) {
      const int r = e / nb, c = e % nb;
      Wj[r * nb + c] = sm.W[r * LDW + c];
    }
    // forward: z = b_j + tprev .* w_{j-1}
    for (int o = threadIdx.x; o < nb * nrhs; o += NT) {
      const int k = o / nb, r = o % nb;
      double v = scr[(long long)k * B.ncell + j * nb + r];
      if (j > 0) v += sm.tprev[r] * scr[(long long)k * B.ncell + (j - 1) * nb + r];
      sm.Z[k * kMaxBlock + r] = v;
    }
    __syncthreads();
    block_gemv(nb, nrhs, sm.W, LDW, sm.Z, scr + (long long)j * nb, B.ncell, nullptr);
  }
  __syncthreads();
}

// Forward sweep with cached inverses (global).
__device__ void forward_sweep(const Geo& g, const Box& B, const double* K, double beta,
                              const double* Wg, double* scr, int nrhs, LocalSmem& sm) {
  const int nb = B.nb;
  for (int j = 0; j < B.nblk; ++j) {
    __syncthreads();
    if (j > 0)
      for (int a = threadIdx.x; a < nb; a += NT) sm.tprev[a] = sm.tnext[a];
    __syncthreads();
    load_block_coefs(g, B, K, beta, j, sm);
    for (int o = threadIdx.x; o < nb * nrhs; o += NT) {
      const int k = o / nb, r = o % nb;
      double v = scr[(long long)k * B.ncell + j * nb + r];
      if (j > 0) v += sm.tprev[r] * scr[(long long)k * B.ncell + (j - 1) * nb + r];
      sm.Z[k * kMaxBlock + r] = v;
    }
    __syncthreads();
    block_gemv(nb, nrhs, Wg + (long long)j * nb * nb, nb, sm.Z, scr + (long long)j * nb, B.ncell,
               nullptr);
  }
  __syncthreads();
}

// Global coordinates of box cell `loc`.
__device__ __forceinline__ void loc_cell(const Box& B, int loc, int c[3]) {
  int u[3];
  box_local(B, loc, u);
  c[0] = B.lo[0] + u[0];
  c[1] = B.lo[1] + u[1];
  c[2] = B.lo[2] + u[2];
}

__device__ __forceinline__ int cell_loc(const Box& B, const int c[3]) {
  const int m0 = B.hi[0] - B.lo[0], m1 = B.hi[1] - B.lo[1];
  return (c[0] - B.lo[0]) + m0 * ((c[1] - B.lo[1]) + m1 * (c[2] - B.lo[2]));
}

__device__ __forceinline__ bool in_box(const Box& B, const int c[3]) {
  return c[0] >= B.lo[0] && c[0] < B.hi[0] && c[1] >= B.lo[1] && c[1] < B.hi[1] &&
         c[2] >= B.lo[2] && c[2] < B.hi[2];
}

// Omega_i extent of subdomain `sub`.
__device__ __forceinline__ void omega_of(const Geo& g, int sub, int lo[3], int hi[3]) {
  int r = sub;
  for (int a = 0; a < 3; ++a) {
    const int Ma = (a < g.d) ? g.M[a] : 1;
    const int ia = r % Ma;
    r /= Ma;
    lo[a] = (a < g.d) ? ia * g.S[a] : 0;
    hi[a] = (a < g.d) ? lo[a] + g.S[a] : 1;
  }
}

__device__ __forceinline__ int neighbor_of(const Geo& g, int sub, int q) {
  const int a = q >> 1, s = q & 1;
  int r = sub, stride = 1, ia = 0;
  for (int b = 0; b < a; ++b) stride *= g.M[b];
  ia = (r / stride) % g.M[a];
  const int t = ia + (s ? 1 : -1);
  if (off_subgrid(g, a, ia, t)) return -1;
  return sub + (s ? stride : -stride);
}

// Enumerate faces of Gamma side q of Omega_i: face t -> inner cell.
__device__ __forceinline__ void gamma_face_cell(const Geo& g, const int lo[3], const int hi[3],
                                                int q, int t, int c[3]) {
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

__device__ __forceinline__ int gamma_nfaces(const Geo& g, int q) {
  const int a = q >> 1;
  int n = 1;
  for (int b = 0; b < g.d; ++b)
    if (b != a) n *= g.S[b];
  return n;
}

// ------------------------------------------------------------------ kernels

__global__ void k_exp(const double* __restrict__ logk, double* __restrict__ K, int n,
                      int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double y = logk[i];
  const double k = exp(y);
  if (!(k > 0.0) || !isfinite(k)) atomicOr(flags, kFlagBadK);
  K[i] = k;
}

__global__ void k_fill(double* p, double v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f(float* p, float v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Steps 1-2 (oversampling problems): factor box, solve all seeds, extract
// u, phi on Gamma_i and the restriction to Omega_i.
__global__ void __launch_bounds__(NT) k_basis(Geo g, const Box* __restrict__ boxes,
                                              const Seed* __restrict__ seeds,
                                              const double* __restrict__ K, double beta,
                                              double* __restrict__ fac, double* __restrict__ scr,
                                              double* __restrict__ Pk, double* __restrict__ tr_u,
                                              double* __restrict__ tr_phi,
                                              double* __restrict__ tr_beta, int* flags,
                                              int factor_only) {
  __shared__ LocalSmem sm;
  const Box B = boxes[blockIdx.x];
  if (threadIdx.x == 0) sm.flag = 0;
  // factor_only (Algorithm 1, Step 6): the factor with the smoothing Robin
  // parameter, no right-hand side
  const int nrhs = factor_only ? 0 : B.nrhs;
  double* S = scr + B.scr;
  // right-hand sides: T^R * seed on the seed's side
  for (long long e = threadIdx.x; e < (long long)nrhs * B.ncell; e += NT) S[e] = 0.0;
  __syncthreads();
  for (int k = 0; k < nrhs; ++k) {
    const Seed sd = seeds[B.seed0 + k];
    const int a = sd.side >> 1, s = sd.side & 1;
    // cells of the box on that side
    int nf = 1;
    for (int b = 0; b < g.d; ++b)
      if (b != a) nf *= (B.hi[b] - B.lo[b]);
    for (int t = threadIdx.x; t < nf; t += NT) {
      int c[3], r = t;
      for (int b = 0; b < 3; ++b) {
        if (b == a) c[b] = s ? B.hi[b] - 1 : B.lo[b];
        else {
          const int m = B.hi[b] - B.lo[b];
          c[b] = B.lo[b] + r % m;
          r /= m;
        }
      }
      int o[3] = {c[0], c[1], c[2]};
      o[a] += s ? 1 : -1;
      const double* Ka = K + kaxis(g, a);
      const double kc = Ka[gcell(g, c)];
      const double bt = robin_beta(g, a, kc, Ka[gcell(g, o)], beta);
      S[(long long)k * B.ncell + cell_loc(B, c)] = robin_T(g, kc, bt) * seed_value(g, sd, B.lo, B.hi, c);
    }
  }
  __syncthreads();
  double* Wg = fac + B.fac;
  factor_forward(g, B, K, beta, Wg, S, nrhs, sm);
  backward_sweep(g, B, K, beta, Wg, S, nrhs, sm);
  // restriction to Omega_i and traces on Gamma_i
  int olo[3], ohi[3];
  omega_of(g, B.sub, olo, ohi);
  const int ncell_o = g.S[0] * g.S[1] * (g.d == 3 ? g.S[2] : 1);
  for (int e = threadIdx.x; e < nrhs * ncell_o; e += NT) {
    const int k = e / ncell_o, t = e % ncell_o;
    int c[3];
    c[0] = olo[0] + t % g.S[0];
    c[1] = olo[1] + (t / g.S[0]) % g.S[1];
    c[2] = (g.d == 3) ? olo[2] + t / (g.S[0] * g.S[1]) : 0;
    Pk[(long long)(B.seed0 + k) * ncell_o + t] = S[(long long)k * B.ncell + cell_loc(B, c)];
  }
  for (int q = 0; q < 2 * g.d; ++q) {
    const int nf = gamma_nfaces(g, q);
    const bool has = neighbor_of(g, B.sub, q) >= 0;
    const int a = q >> 1, s = q & 1;
    for (int e = threadIdx.x; e < nrhs * nf; e += NT) {
      const int k = e / nf, t = e % nf;
      const long long oidx = (long long)(B.seed0 + k) * g.gstride + g.gside_off[q] + t;
      if (!has) {
        tr_u[oidx] = 0.0;
        tr_phi[oidx] = 0.0;
        continue;
      }
      int c[3], o[3];
      gamma_face_cell(g, olo, ohi, q, t, c);
      o[0] = c[0]; o[1] = c[1]; o[2] = c[2];
      o[a] += s ? 1 : -1;
      const double kc = K[kaxis(g, a) + gcell(g, c)], ko = K[kaxis(g, a) + gcell(g, o)];
      const double Pc = S[(long long)k * B.ncell + cell_loc(B, c)];
      double u;
      if (in_box(B, o)) {
        const double T = g.area * kharm(kc, ko) / g.h;
        u = T * (Pc - S[(long long)k * B.ncell + cell_loc(B, o)]) / g.area;
      } else {
        const Seed sd = seeds[B.seed0 + k];
        const double lam = (sd.side == q) ? seed_value(g, sd, B.lo, B.hi, c) : 0.0;
        const double bt = robin_beta(g, a, kc, ko, beta);
        u = robin_T(g, kc, bt) * (Pc - lam) / g.area;
      }
      const double pi = Pc - u * g.h / (2.0 * kc);
      const double bt = robin_beta(g, a, kc, ko, beta);
      tr_u[oidx] = u;
      tr_phi[oidx] = -bt * u + pi;
      if (k == 0) tr_beta[(long long)B.sub * g.gstride + g.gside_off[q] + t] = bt;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && sm.flag) atomicOr(flags, sm.flag);
}

// Right-hand side of the physical data (source, pressure and velocity
// boundary conditions) for box B into S (one vector).
__device__ void physical_rhs(const Geo& g, const Box& B, const double* K, const double* f,
                             const double* bcv, double* S) {
  for (int loc = threadIdx.x; loc < B.ncell; loc += NT) {
    int c[3];
    loc_cell(B, loc, c);
    const int ci = gcell(g, c);
    double b = f ? f[ci] * g.vol : 0.0;
    for (int a = 0; a < g.d; ++a)
      for (int s = 0; s < 2; ++s) {
        const int t = c[a] + (s ? 1 : -1);
        if (!off_domain(g, a, c[a], t)) continue;
        const int side = 2 * a + s;
        const double val = bcv[g.bc_off[side] + bface_index(g, c, a)];
        if (g.bc_type[side]) b += 2.0 * K[kaxis(g, a) + ci] * g.area / g.h * val;
        else b -= g.area * val;
      }
    S[loc] = b;
  }
}

// Step 4: particular problem on Omega_i (zero Robin data on Gamma_i).
__global__ void __launch_bounds__(NT) k_particular(Geo g, const Box* __restrict__ boxes,
                                                   const double* __restrict__ K,
                                                   const double* __restrict__ f,
                                                   const double* __restrict__ bcv, double beta,
                                                   double* __restrict__ fac,
                                                   double* __restrict__ scr,
                                                   double* __restrict__ pbar,
                                                   double* __restrict__ ubar,
                                                   double* __restrict__ pibar, int* flags) {
  __shared__ LocalSmem sm;
  const Box B = boxes[blockIdx.x];
  if (threadIdx.x == 0) sm.flag = 0;
  double* S = scr + B.scr;
  physical_rhs(g, B, K, f, bcv, S);
  __syncthreads();
  double* Wg = fac + B.fac;
  factor_forward(g, B, K, beta, Wg, S, 1, sm);
  backward_sweep(g, B, K, beta, Wg, S, 1, sm);
  for (int t = threadIdx.x; t < B.ncell; t += NT) pbar[(long long)B.sub * B.ncell + t] = S[t];
  for (int q = 0; q < 2 * g.d; ++q) {
    const int nf = gamma_nfaces(g, q);
    const bool has = neighbor_of(g, B.sub, q) >= 0;
    const int a = q >> 1, s = q & 1;
    for (int t = threadIdx.x; t < nf; t += NT) {
      const long long oidx = (long long)B.sub * g.gstride + g.gside_off[q] + t;
      if (!has) {
        ubar[oidx] = 0.0;
        pibar[oidx] = 0.0;
        continue;
      }
      int c[3], o[3];
      gamma_face_cell(g, B.lo, B.hi, q, t, c);
      o[0] = c[0]; o[1] = c[1]; o[2] = c[2];
      o[a] += s ? 1 : -1;
      const double* Ka = K + kaxis(g, a);
      const double kc = Ka[gcell(g, c)];
      const double bt = robin_beta(g, a, kc, Ka[gcell(g, o)], beta);
      const double u = robin_T(g, kc, bt) * (S[cell_loc(B, c)] - 0.0) / g.area;
      ubar[oidx] = u;
      pibar[oidx] = bt * u;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && sm.flag) atomicOr(flags, sm.flag);
}

// Robin data lambda = -beta u.n + pi on a Robin face of box B (outward
// normal of the box), from the current global state (Section 3, item 3).
__device__ __forceinline__ double smooth_lambda(const Geo& g, const Box& B, const double* K,
                                                const double* p, const double* gflux, double beta,
                                                const int c[3], int a, int s) {
  int o[3] = {c[0], c[1], c[2]};
  o[a] += s ? 1 : -1;
  const int ci = gcell(g, c), oi = gcell(g, o);
  const double kc = K[kaxis(g, a) + ci], ko = K[kaxis(g, a) + oi];
  const double bt = robin_beta(g, a, kc, ko, beta);
  if (g.l > 0) {
    const double u = g.area * kharm(kc, ko) / g.h * (p[ci] - p[oi]) / g.area;
    const double pi = p[ci] - u * g.h / (2.0 * kc);
    return -bt * u + pi;
  }
  // no overlap: the neighbour's own flux and pressure trace on the shared face
  const int q = 2 * a + s;
  const int j = neighbor_of(g, B.sub, q);
  int jlo[3], jhi[3];
  omega_of(g, j, jlo, jhi);
  const int t = side_face_index(g, jlo, jhi, o, a);
  const double uj = gflux[(long long)j * g.gstride + g.gside_off[q ^ 1] + t];
  const double pij = p[oi] - uj * g.h / (2.0 * ko);
  return bt * uj + pij;
}

// Steps 6-7: one color phase of the smoothing sweep (FP64 factors).
__global__ void __launch_bounds__(NT) k_smooth(Geo g, const Box* __restrict__ boxes,
                                               const int* __restrict__ members,
                                               const double* __restrict__ K,
                                               const double* __restrict__ f,
                                               const double* __restrict__ bcv, double beta,
                                               const double* __restrict__ fac,
                                               double* __restrict__ scr, double* __restrict__ p,
                                               double* __restrict__ gflux) {
  __shared__ LocalSmem sm;
  const Box B = boxes[members[blockIdx.x]];
  double* S = scr + B.scr;
  physical_rhs(g, B, K, f, bcv, S);
  __syncthreads();
  // Robin contributions
  for (int loc = threadIdx.x; loc < B.ncell; loc += NT) {
    int c[3];
    loc_cell(B, loc, c);
    double add = 0.0;
    for (int a = 0; a < g.d; ++a)
      for (int s = 0; s < 2; ++s) {
        if (face_kind(g, B, c, a, s) != kFaceRobin) continue;
        int o[3] = {c[0], c[1], c[2]};
        o[a] += s ? 1 : -1;
        const double kc = K[kaxis(g, a) + gcell(g, c)];
        const double bt = robin_beta(g, a, kc, K[kaxis(g, a) + gcell(g, o)], beta);
        add += robin_T(g, kc, bt) * smooth_lambda(g, B, K, p, gflux, beta, c, a, s);
      }
    S[loc] += add;
  }
  __syncthreads();
  const double* Wg = fac + B.fac;
  forward_sweep(g, B, K, beta, Wg, S, 1, sm);
  backward_sweep(g, B, K, beta, Wg, S, 1, sm);
  // Gamma fluxes of Omega_i from the box solution (before p is overwritten:
  // for l = 0 they need lambda, which reads the neighbour, not Omega_i)
  int olo[3], ohi[3];
  omega_of(g, B.sub, olo, ohi);
  for (int q = 0; q < 2 * g.d; ++q) {
    if (neighbor_of(g, B.sub, q) < 0) continue;
    const int nf = gamma_nfaces(g, q);
    const int a = q >> 1, s = q & 1;
    for (int t = threadIdx.x; t < nf; t += NT) {
      int c[3], o[3];
      gamma_face_cell(g, olo, ohi, q, t, c);
      o[0] = c[0]; o[1] = c[1]; o[2] = c[2];
      o[a] += s ? 1 : -1;
      const double kc = K[kaxis(g, a) + gcell(g, c)], ko = K[kaxis(g, a) + gcell(g, o)];
      const double xc = S[cell_loc(B, c)];
      double u;
      if (in_box(B, o)) {
        u = g.area * kharm(kc, ko) / g.h * (xc - S[cell_loc(B, o)]) / g.area;
      } else {
        const double lam = smooth_lambda(g, B, K, p, gflux, beta, c, a, s);
        u = robin_T(g, kc, robin_beta(g, a, kc, ko, beta)) * (xc - lam) / g.area;
      }
      gflux[(long long)B.sub * g.gstride + g.gside_off[q] + t] = u;
    }
  }
  __syncthreads();
  const int ncell_o = g.S[0] * g.S[1] * (g.d == 3 ? g.S[2] : 1);
  for (int t = threadIdx.x; t < ncell_o; t += NT) {
    int c[3];
    c[0] = olo[0] + t % g.S[0];
    c[1] = olo[1] + (t / g.S[0]) % g.S[1];
    c[2] = (g.d == 3) ? olo[2] + t / (g.S[0] * g.S[1]) : 0;
    p[gcell(g, c)] = S[cell_loc(B, c)];
  }
}

}  // namespace

hipError_t launch_exp(const double* logk, double* K, int n, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_exp, dim3((n + 255) / 256), dim3(256), 0, s, logk, K, n, flags);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, double v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f(float* p, float v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_basis(const Geo& g, const Box* boxes, int nbox, const Seed* seeds,
                        const double* K, double beta, double* fac, double* scr, double* Pk,
                        double* tr_u, double* tr_phi, double* tr_beta, int* flags,
                        hipStream_t s, int factor_only) {
  if (nbox <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_basis, dim3(nbox), dim3(NT), 0, s, g, boxes, seeds, K, beta, fac, scr, Pk,
                     tr_u, tr_phi, tr_beta, flags, factor_only);
  return hipGetLastError();
}

hipError_t launch_particular(const Geo& g, const Box* boxes, int nbox, const double* K,
                             const double* f, const double* bcv, double beta, double* fac,
                             double* scr, double* pbar, double* ubar, double* pibar, int* flags,
                             hipStream_t s) {
  if (nbox <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_particular, dim3(nbox), dim3(NT), 0, s, g, boxes, K, f, bcv, beta, fac,
                     scr, pbar, ubar, pibar, flags);
  return hipGetLastError();
}

hipError_t launch_smooth(const Geo& g, const Box* boxes, const int* members, int nmem,
                         const double* K, const double* f, const double* bcv, double beta,
                         const double* fac, const float* fac32, const double* dscale, double* scr,
                         double* p, double* gflux, int precision, double tol, int max_refine,
                         int* iters, double* resid, int* flags, hipStream_t s) {
  if (nmem <= 0) return hipSuccess;
  (void)fac32; (void)dscale; (void)precision; (void)tol; (void)max_refine; (void)iters;
  (void)resid; (void)flags;
  hipLaunchKernelGGL(k_smooth, dim3(nmem), dim3(NT), 0, s, g, boxes, members, K, f, bcv, beta, fac,
                     scr, p, gflux);
  return hipGetLastError();
}

}  // namespace mrcm
