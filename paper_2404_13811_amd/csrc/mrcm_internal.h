// Internal declarations shared by the host runtime and the HIP kernels of
// the MRCM-OS library.  Nothing here is part of the public ABI (mrcm.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

namespace mrcm {

constexpr int kMaxBlock = 64;       // largest dense block (cells of one line / plane)
constexpr int kLocalThreads = 256;  // threads per local-solve workgroup
constexpr int kMaxRhs = 64;         // right-hand sides per box in one launch

// Flags raised by kernels (bit mask in device memory).
enum : int { kFlagNotPD = 1, kFlagSingular = 2, kFlagNoConv = 4, kFlagBadK = 8, kFlagBandOverflow = 16 };

// Geometry and discretisation parameters, passed to every kernel by value.
struct Geo {
  int d;
  int n[3];        // cells per axis (1 for unused axes)
  int S[3];        // cells per subdomain per axis
  int M[3];        // subdomains per axis
  int l;           // oversampling width
  int nsub;
  int ncells;
  int bc_type[6];  // 0 Neumann, 1 Dirichlet
  int bc_off[6];   // offset of each side's face values in the bc array
  int beta_mode;   // 0 alpha, 1 constant
  int neumann;     // no pressure boundary anywhere
  int nfaceg;      // faces per Gamma side (S^(d-1)), same for every side when S is cubic
  int gside_off[6];// offset of side q within one subdomain's Gamma-face block
  int gstride;     // faces per subdomain over all 2d sides
  // batches of 2-D problems: the members are stacked along axis 1, cut
  // cells (mcut subdomain rows) each; nothing couples cells or subdomains
  // across a cut, which bounds each member like the domain boundary
  // (0: one problem)
  int cut, mcut;
  // permeability entries per cell: 1 (scalar K) or d (diagonal tensor,
  // component-major: the entry of axis a of cell c at K[a * ncells + c])
  int kc;
  double h, area, vol;
};

// Offset of axis a's permeability entries (0 for scalar K).
__host__ __device__ inline long long kaxis(const Geo& g, int a) {
  return g.kc > 1 ? (long long)a * g.ncells : 0;
}

// Moving from coordinate `from` to `to` along axis a leaves the domain (or
// the batch member).
__host__ __device__ inline bool off_domain(const Geo& g, int a, int from, int to) {
  return to < 0 || to >= g.n[a] || (a == 1 && g.cut > 0 && to / g.cut != from / g.cut);
}

// The subdomain at coordinate `to` along axis a is no neighbour of the one
// at `from` (outside the grid of subdomains or across a batch cut).
__host__ __device__ inline bool off_subgrid(const Geo& g, int a, int from, int to) {
  return to < 0 || to >= g.M[a] || (a == 1 && g.mcut > 0 && to / g.mcut != from / g.mcut);
}

// One local box: an oversampled region (basis functions, smoothing) or a
// subdomain (particular problem).  Cells are ordered x fastest; blocks are
// the cells sharing the last-axis coordinate.
struct Box {
  int lo[3], hi[3];
  int sub;
  int nb, nblk, ncell;
  int nrhs;
  int seed0;          // first global seed index (basis boxes)
  long long fac;      // element offset of the cached block inverses
  long long scr;      // element offset of this box's right-hand-side scratch
};

// Seed Robin data on one side of an oversampled box, and (with the same
// encoding, measured on the subdomain) a test function of M_H / V_H.
struct Seed {
  int side;   // 0..2d-1
  int kind;   // 0 constant, 1 linear along tangential axis `axis`, 2 fine indicator
  int axis;
  int face;   // fine: face index on the side (x-fastest over tangential axes)
};

// A coarse interface Gamma_ij, i < j, normal along `axis`.
struct Iface {
  int i, j, axis;
  int row0;     // first row of its 2p equations
  int nbasis;   // p
  int basis0;   // index of its first test function in the basis array
};

// One batched product of the cyclic reduction: the matrix at pool offset c
// := [matrix at c0] + al1 * a1 * b1 [+ al2 * a2 * b2]  (element offsets of
// n x n operands with the launch's leading dimension; < 0 drops a term).
struct BcrGemm {
  long long c, c0, a1, b1, a2, b2;
  double al1, al2;
  // column window of a windowed rectangular product (launch_rect_gemm_win):
  // columns [wc0, wc1) and column wcx (< 0: none) of C, rounded out to
  // whole tiles; the other columns are neither read from B nor written
  int wc0 = 0, wc1 = 0, wcx = -1, pad = 0;
};
// Vector form: vector y := [vector y0] + al1 * block a1 * vector x1 [+ ...].
struct BcrGemv {
  int y, y0, a1, x1, a2, x2;
  double al1, al2;
};

// ---------------------------------------------------------------- launchers
// local problems (local.hip)
hipError_t launch_exp(const double* logk, double* K, int n, int* flags, hipStream_t s);
hipError_t launch_fill(double* p, double v, long long n, hipStream_t s);
hipError_t launch_fill_f(float* p, float v, long long n, hipStream_t s);
// factor_only != 0: factor the boxes with beta and solve nothing (Algorithm
// 1, Step 6: the smoothing factor when its Robin parameter differs)
hipError_t launch_basis(const Geo& g, const Box* boxes, int nbox, const Seed* seeds,
                        const double* K, double beta, double* fac, double* scr,
                        double* Pk, double* tr_u, double* tr_phi, double* tr_beta,
                        int* flags, hipStream_t s, int factor_only = 0);
hipError_t launch_particular(const Geo& g, const Box* boxes, int nbox, const double* K,
                             const double* f, const double* bcv, double beta, double* fac,
                             double* scr, double* pbar, double* ubar, double* pibar,
                             int* flags, hipStream_t s);
hipError_t launch_factor32(const Geo& g, const Box* boxes, int nbox, const double* K,
                           double beta, float* fac32, double* dscale, int* flags, hipStream_t s);
hipError_t launch_basis32(const Geo& g, const Box* boxes, int nbox, const Seed* seeds,
                          const double* K, double beta, const float* fac32, const double* dscale,
                          double* scr, double* Pk, double* tr_u, double* tr_phi, double* tr_beta,
                          double tol, int max_refine, int* iters, double* resid, int* flags,
                          hipStream_t s);
hipError_t launch_particular32(const Geo& g, const Box* boxes, int nbox, const double* K,
                               const double* f, const double* bcv, double beta,
                               const float* fac32, const double* dscale, double* scr,
                               double* pbar, double* ubar, double* pibar, double tol,
                               int max_refine, int* iters, double* resid, int* flags,
                               hipStream_t s);
hipError_t launch_smooth(const Geo& g, const Box* boxes, const int* members, int nmem,
                         const double* K, const double* f, const double* bcv, double beta,
                         const double* fac, const float* fac32, const double* dscale,
                         double* scr, double* p, double* gflux, int precision, double tol,
                         int max_refine, int* iters, double* resid, int* flags, hipStream_t s);

// one-wavefront-per-box 2-D kernels (local_wave.hip), blocks of <= 32 cells
size_t wave_lds_bytes(int m0, int m1, int nrhs, int kc);
// LDS of a two-wave basis box of k_local_w
size_t wave_basis_lds_bytes(int m0, int m1, int nrhs, int kc);
size_t wave_smooth_lds_bytes(int m0, int m1, int kc);
// Steps 1-2 (oversampled boxes obox) and Step 4 (subdomain boxes pbox, one
// or two per workgroup) in one launch; lds_part = LDS of one subdomain box,
// lds >= the basis boxes' need and lds_part (two per workgroup when lds
// holds two and there are more than twice as many boxes as CUs).
// The kernel reads log K and writes K = exp(log K) (each subdomain its own
// cells; kFlagBadK where K is not finite and positive).  fac: forward
// inverses below the meeting block of every oversampled box; fact (not
// null): backward inverses above it and the meeting block, same layout.
hipError_t launch_local_w(const Geo& g, const Box* obox, const Box* pbox, int nbox,
                          const Seed* seeds, const double* logK, double* K, const double* f,
                          const double* bcv,
                          double beta, double* fac, double* tcoup, double* facp, double* tcp,
                          double* Pk, double* tr_u, double* tr_phi, double* tr_beta, double* pbar,
                          double* ubar, double* pibar, double* fact, int* flags, size_t lds,
                          size_t lds_part, hipStream_t s);
// Algorithm 1, Step 6: the oversampled boxes factored again with the
// smoothing Robin parameter into fac (forward inverses) and fact (backward
// inverses, meeting block), the layout k_local_w writes; lds as its basis
// boxes with no right-hand side
hipError_t launch_factor_w(const Geo& g, const Box* obox, int nbox, const double* logK,
                           double beta, double* fac, double* fact, int* flags, size_t lds,
                           hipStream_t s);
hipError_t launch_smooth_w(const Geo& g, const Box* boxes, int nmem,
                           const double* K, const double* f, const double* bcv, double beta,
                           const double* fac, const double* fact, const double* tcoup, double* scr,
                           double* p, double* gflux, size_t lds, int nt, hipStream_t s);
// colour phases of the smoothing sweep: boxes of colour c are
// members[off[c] .. off[c+1])
struct SmoothPhases {
  int off[9];
  int ncol;
};
// nphase colour phases (phase k has colour k % ncol) in one cooperative
// launch with a grid barrier between phases: as many workgroups as fit on
// the device at once (at most the largest colour's box count, and at most
// max_groups when that is > 0), each looping over its share of a phase's
// boxes; hipErrorNotSupported when the device has no cooperative launch,
// hipErrorCooperativeLaunchTooLarge when not one workgroup fits (nothing is
// launched in either case)
hipError_t launch_smooth_grid(const Geo& g, const Box* boxes, const SmoothPhases& ph, int nphase, const double* K, const double* f,
                              const double* bcv, double beta, const double* fac, const double* fact,
                              const double* tcoup, double* p, double* gflux, size_t lds, int nt,
                              int max_groups, hipStream_t s);

// one-wavefront-per-box 3-D kernels (local3.hip), plane blocks of <= 64 cells
size_t box3_lds_bytes(int m0, int m1, int m2, int nrhs, int kc);
// wavefronts per box for plane blocks of nb cells (1, 2 or 4)
int box3_waves(int nb);
// Steps 1-2 (factor_only: Step 6) on oversampled boxes; reads log K
hipError_t launch_basis3(const Geo& g, const Box* boxes, int nbox, const Seed* seeds,
                         const double* logK, double beta, double* fac, double* Pk, double* tr_u,
                         double* tr_phi, double* tr_beta, int factor_only, int* flags, size_t lds,
                         int nw, hipStream_t s);
// Step 4 on the subdomains; writes K = exp(log K) (kFlagBadK where not
// finite and positive)
hipError_t launch_particular3(const Geo& g, const Box* boxes, int nbox, const double* logK, double* K,
                              const double* f, const double* bcv, double beta, double* fac,
                              double* pbar, double* ubar, double* pibar, int* flags, size_t lds, int nw,
                              hipStream_t s);
// one colour phase of the smoothing sweep (boxes in colour order)
hipError_t launch_smooth3(const Geo& g, const Box* boxes, int nmem, const double* K, const double* f,
                          const double* bcv, double beta, const double* fac, double* p, double* gflux,
                          size_t lds, int nw, hipStream_t s);

// The same 3-D local problems in the FP32 form (local3f.hip): FP32 plane
// inverses of the diagonally scaled box matrix, FP64 refinement of every
// solve to the componentwise backward error tol (at most max_refine + 1
// FP32 solves; the most taken and the largest final error to iters and
// resid).  LDS bytes of a box with nrhs solutions and nbv FP64 right-hand
// sides stored.  Smoothing: a box holds the inverses of its first `cached`
// planes (8, 4, 2 or 0) in registers across its refinement sweeps and reads
// the others for every sweep.
size_t box3f_lds_bytes(int m0, int m1, int m2, int nrhs, int nbv, int kc);
// seeds an FP32 basis box solves at a time (after its factor)
constexpr int kSeedBatch3f = 3;
hipError_t launch_basis3f(const Geo& g, const Box* boxes, int nbox, const Seed* seeds, const double* logK,
                          double beta, float* fac32, double* Pk, double* tr_u, double* tr_phi,
                          double* tr_beta, int factor_only, double tol, int max_refine, int* iters,
                          unsigned long long* resid, int* flags, size_t lds, int nw, hipStream_t s);
hipError_t launch_particular3f(const Geo& g, const Box* boxes, int nbox, const double* logK, double* K,
                               const double* f, const double* bcv, double beta, float* facp32,
                               double* pbar, double* ubar, double* pibar, double tol, int max_refine,
                               int* iters, unsigned long long* resid, int* flags, size_t lds, int nw,
                               hipStream_t s);
hipError_t launch_smooth3f(const Geo& g, const Box* boxes, int nmem, const double* K, const double* f,
                           const double* bcv, double beta, const float* fac32, double* p, double* gflux,
                           double tol, int max_refine, int* iters, unsigned long long* resid, int* flags,
                           size_t lds, int nw, int cached, hipStream_t s);

// FP32 factors with FP64 iterative refinement (local_wave32.hip)
size_t wave32_lds_bytes(int m0, int m1, int nrhs, int nbrhs, int kc);
size_t wave32_smooth_lds_bytes(int m0, int m1, int kc);
hipError_t launch_local32_w(const Geo& g, const Box* obox, const Box* pbox, int nbox,
                            const Seed* seeds, const double* K, const double* f, const double* bcv,
                            double beta, float* fac32, float* facp32, double* Pk, double* tr_u,
                            double* tr_phi, double* tr_beta, double* pbar, double* ubar,
                            double* pibar, double tol, int max_refine, int* iters,
                            unsigned long long* resid, int* flags, size_t lds, hipStream_t s);
// Step 6 in the FP32 form: FP32 factors of the scaled oversampled boxes
// with the smoothing Robin parameter (K must hold exp(log K))
hipError_t launch_factor32_w(const Geo& g, const Box* obox, int nbox, const double* K, double beta,
                             float* fac32, int* iters, unsigned long long* resid, int* flags,
                             size_t lds, hipStream_t s);
hipError_t launch_smooth32_w(const Geo& g, const Box* boxes, int nmem,
                             const double* K, const double* f, const double* bcv, double beta,
                             const float* fac32, double* p, double* gflux, double tol,
                             int max_refine, int* iters, unsigned long long* resid, int* flags,
                             size_t lds, int nt, hipStream_t s);

// interface system (iface.hip)
// Where the moments go when the interface system is solved by block cyclic
// reduction: equation row / unknown col to (layer, position), the layer
// blocks [D | L | U] (M layers, bp x bp each) and right-hand sides.  pool
// NULL: the row band AB and rhs.
// With dst set (the two-level solver), entry e of equation row `row` (e
// counting the seeds of the lower subdomain, then those of the higher one)
// goes to pool[dst[row * dstw + e]] (skipped where < 0) and the row's
// right-hand side to pool[rdst[row]].
struct BcrMap {
  const int* row_lvl = nullptr;
  const int* row_loc = nullptr;
  const int* col_lvl = nullptr;
  const int* col_loc = nullptr;
  int M = 0, bp = 0;
  double* pool = nullptr;
  double* vec = nullptr;
  const long long* dst = nullptr;
  const long long* rdst = nullptr;
  int dstw = 0;
};
hipError_t launch_moments(const Geo& g, const Iface* ifc, int nifc, int nrow_max, const Seed* basis,
                          const int* seed_off, const double* tr_u, const double* tr_phi,
                          const double* tr_beta, const double* ubar, const double* pibar,
                          double* AB, int ldab, int kl, int ku, double* rhs, hipStream_t s,
                          const BcrMap* bm = nullptr);
hipError_t launch_bandlu_solve(double* AB, int ldab, int n, int kl, int ku, double* rhs,
                               double* x, int* ipiv, int* flags, hipStream_t s);
hipError_t launch_combine(const Geo& g, const int* seed_off, const double* X, const double* Pk,
                          const double* tr_u, const double* pbar, const double* ubar,
                          double* p, double* gflux, hipStream_t s);

// block cyclic reduction of the interface system (bcr.hip)
constexpr int kBcrMaxBlock = 256;  // layer block (two-by-two inverse above kBcrInvMax)
constexpr int kBcrInvMax = 128;    // largest block one Gauss-Jordan workgroup inverts
hipError_t launch_bcr_inv(double* pool, const long long* offs, const int* npiv, int nblk, int n,
                          int ld, int* flags, hipStream_t s);
hipError_t launch_bcr_gemm(double* pool, const BcrGemm* tasks, int ntask, int n, int ld, hipStream_t s);
// independent products and block-vector products of one reduction step in
// one launch (no vector task may read a block the products write)
hipError_t launch_bcr_gemm_gemv(double* pool, double* vec, const BcrGemm* gtasks, int ngemm,
                               const BcrGemv* vtasks, int ngemv, int n, int ld, int bp,
                               hipStream_t s);
hipError_t launch_bcr_gemv(const double* pool, double* vec, const BcrGemv* tasks, int ntask, int bp,
                           hipStream_t s);
hipError_t launch_bcr_gather(const double* xv, const int* col_lvl, const int* col_loc, int n, int bp,
                             double* X, hipStream_t s);
// zero pool and right-hand sides, identity on the padded diagonals of D
hipError_t launch_bcr_init(double* pool, double* vec, const int* lsize, int M, int bp, hipStream_t s);

// two-level interface solver (bcr_rect.hip, iface_lsc.cpp)
struct RectShape {
  int m, n, k;       // C: m x n, A: m x k, B: k x n (multiples of 32)
  int lda, ldb, ldc;
};
// C = [C0] + al1 A1 B1 [+ al2 A2 B2], offsets into one base array (BcrGemm)
hipError_t launch_rect_gemm(double* base, const BcrGemm* tasks, int ntask, const RectShape& S,
                            hipStream_t s);
// products restricted to their column windows (32-column tiles); maxnt:
// the largest number of column tiles of a task's window
hipError_t launch_rect_gemm_win(double* base, const BcrGemm* tasks, int ntask, const RectShape& S,
                                int maxnt, hipStream_t s);
// two independent groups of products with the same k in one launch
hipError_t launch_rect_gemm2(double* base, const BcrGemm* ta, int na, const RectShape& SA,
                             const BcrGemm* tb, int nb, const RectShape& SB, hipStream_t s);
// Runs of zeros: nrep runs of len doubles at base + off, off + stride, ...
// launch_fill_ones: the runs, then base[ones[i]] = 1.
struct ZeroRun {
  long long off, len, stride, nrep;
};
hipError_t launch_fill_ones(double* base, const ZeroRun* runs, int nruns, const long long* ones,
                            long long nones, hipStream_t s);
// One row of the reduced (gap) system: its cross entries (values at
// base[cval + e], stacked-solution rows ypos[yidx + e], < 0: none) applied
// to the inner solution of its source layer (base[ybase + row * ldy + c]),
// column c going where cmap[cm + c] sends it: -2 (the right-hand side) to
// base[rhs], j in [0, ml) (the j-th lower coupling) to base[dst0 + j],
// ml + j (the j-th upper coupling) to base[dst1 + j]; -1 (unused) and
// dst < 0 are dropped.
struct LscRow {
  long long cval, yidx, ybase, rhs, dst0, dst1;
  int cm, ml, ldy, pad;
};
hipError_t launch_lsc_outer_rows(double* base, const LscRow* rows, const long long* ypos,
                                 const int* cmap, int nrow, int ncol, int width, hipStream_t s);
// Back substitution of one interface unknown: its inner solution row at
// base[xrow] (the column of its layer's j-th coupling at icol[cm + j]: the
// ml couplings of s, then the mu of t; the right-hand side at column rc)
// against the reduced solution (s at base[sofs], t at base[tofs]; < 0:
// none).
struct LscCol {
  long long xrow, sofs, tofs;
  int ml, mu, cm, pad;
};
hipError_t launch_lsc_back(const double* base, const LscCol* cols, const int* icol, int n, int rc,
                           double* X, hipStream_t s);

// The two-level solver's plan and device state (iface_lsc.cpp).  seeds_per_side:
// per subdomain and side (6 entries each) its number of seeds.  Returns
// null with *err (and *herr for a failed HIP call) when the grid does not
// suit it.
struct Lsc;
Lsc* lsc_create(const Geo& g, const std::vector<Iface>& ifc, const std::vector<int>& seed_off,
                const std::vector<int>& seeds_per_side, int nX, std::string* err, hipError_t* herr);
void lsc_destroy(Lsc* L);
// zero the workspace and set its identity and unit entries (before the moments)
hipError_t lsc_prepare(Lsc* L, hipStream_t s);
// where the moments of the interface equations go
BcrMap lsc_map(const Lsc* L);
// inner reductions, reduced system, back substitution into X
hipError_t lsc_solve(Lsc* L, double* X, int* flags, hipStream_t s);
double lsc_bytes(const Lsc* L);
// S, Mi, inner block, right-hand sides, gaps, gap block
void lsc_shape(const Lsc* L, int* out);

// adjoint (adjoint.hip): reverse mode of the 2-D one-wave-per-box path.
// The FP32 form takes its cached FP32 factors of the scaled matrices and
// refinement settings from an Adj32 (launchers: null for the FP64 form).
struct Adj32 {
  const float* fac;  // FP32 block inverses (smoothing / seed boxes, or particular boxes)
  double tol;
  int max_refine;
  int* iters;
  unsigned long long* resid;
  int* flags;
};
size_t adj_smooth_lds_bytes(int m0, int m1, bool f32);
size_t adj_basis_lds_bytes(int m0, int m1, int nrhs, bool f32);
size_t adj_part_lds_bytes(int m0, int m1, bool f32);
hipError_t launch_adj_out(const Geo& g, const double* K, const double* p, const double* bcv,
                          const double* dJdp, const double* dJdf, double* meanp, double* pb,
                          double* gfb, double* Kb, hipStream_t s);
hipError_t launch_adj_smooth(const Geo& g, const Box* boxes, const int* members, int nmem,
                             const double* K, const double* f, const double* bcv, double beta,
                             const double* fac, const double* fact, const double* tcoup,
                             const Adj32* f32, const double* p_in, const double* gf_in, double* pb,
                             double* gfb, double* Kb, size_t lds, hipStream_t s);
hipError_t launch_adj_combine(const Geo& g, const int* seed_sub, int nX, const double* X,
                              const double* Pk, const double* tr_u, const double* pb,
                              const double* gfb, double* Xb, double* tr_ub, hipStream_t s);
hipError_t launch_adj_moments(const Geo& g, const Iface* ifc, int nifc, const Seed* basis,
                              const int* seed_off, const double* X, const double* nu,
                              const double* tr_u, const double* tr_beta, double* tr_ub,
                              double* tr_phib, double* tr_betab, double* ubarb, double* pibarb,
                              hipStream_t s);
hipError_t launch_adj_basis(const Geo& g, const Box* boxes, int nbox, const Seed* seeds,
                            const double* K, double beta, const double* fac, const double* fact,
                            const Adj32* f32, const double* X, const double* pb, const double* tr_u,
                            const double* tr_ub, const double* tr_phib, const double* tr_betab,
                            double* Kb, size_t lds, hipStream_t s);
hipError_t launch_adj_particular(const Geo& g, const Box* boxes, int nbox, const double* K,
                                 const double* bcv, double beta, const double* fac, const Adj32* f32,
                                 const double* pbar, const double* pb, const double* ubarb,
                                 const double* pibarb, double* Kb, size_t lds, hipStream_t s);
hipError_t launch_adj_logk(const double* K, const double* Kb, int n, double* out, hipStream_t s);
hipError_t launch_bcr_scatter_t(const double* RB, const double* rhs, int n, int kl, int ku,
                                const int* row_lvl, const int* row_loc, const int* col_lvl,
                                const int* col_loc, int M, int bp, double* pool, double* vec,
                                hipStream_t s);
hipError_t launch_bcr_gather_t(const double* xv, const int* row_lvl, const int* row_loc, int n, int bp,
                               double* out, hipStream_t s);

// conservation and continuity measures of a state (balance.hip)
constexpr int kBalParts = 9;  // max |r_c|, max sum |e||u|, sum f h^d, outflow of 6 sides
// per-cell mass-balance residual (res may be null) and the kBalParts
// quantities into out (partial: cell_balance_blocks(g) * kBalParts doubles)
hipError_t launch_cell_balance(const Geo& g, const double* K, const double* p, const double* gflux,
                               const double* bcv, const double* f, double* res, double* partial,
                               int max_blocks, double* out, hipStream_t s);
int cell_balance_blocks(const Geo& g);
// jump moments of every interface row (mom may be null), largest relative
// flux / pressure jump into jmax[0] / jmax[1] (bits of non-negative
// doubles, max-accumulated: clear them first); tol > 0 raises
// kFlagSingular where a row's relative jump exceeds tol
// The terms of the interface equations, for a componentwise backward
// error (all null: magnitudes of the state's values instead)
struct JumpTerms {
  const double* X = nullptr;
  const int* seed_off = nullptr;
  const double* tr_u = nullptr;
  const double* tr_phi = nullptr;
  const double* tr_beta = nullptr;
  const double* ubar = nullptr;
  const double* pibar = nullptr;
};
hipError_t launch_jumps(const Geo& g, const Iface* ifc, int nifc, const Seed* basis, const double* K,
                        const double* p, const double* gflux, double* mom,
                        unsigned long long* jmax, double tol, int* flags, hipStream_t s,
                        const JumpTerms* terms = nullptr);
// Device address of the static scratch array of mrcm_get_balance_static
// on the current device (kStaticScratchDoubles doubles; looked up once per
// device, then cached)
constexpr int kStaticScratchDoubles = 1 << 16;
constexpr int kMaxDevices = 64;
hipError_t static_scratch(double** ptr);
// relative L2 distance: out[0] = sum (a - b)^2 and out[1] = sum b^2 over
// n values, deterministic (partial: 2 * 256 doubles)
hipError_t launch_sq_dist(const double* a, const double* b, long long n, double* partial,
                          double* out, hipStream_t s);

// outputs (outputs.hip)
hipError_t launch_pressure_out(const Geo& g, const double* p, double* out, double* partial,
                               hipStream_t s);
// pressure (shifted to zero mean for pure-Neumann problems) and face
// velocities: two launches instead of three
hipError_t launch_solution_out(const Geo& g, const double* K, const double* p, const double* gflux,
                               const double* bcv, double* p_out, double* flux_out, double* partial,
                               hipStream_t s);
hipError_t launch_flux_out(const Geo& g, const double* K, const double* p, const double* gflux,
                           const double* bcv, double* out, hipStream_t s);

}  // namespace mrcm
