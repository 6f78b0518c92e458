// Host runtime of the MRCM-OS library: context state machine, partition
// planning (subdomains, oversampled boxes, seeds, interfaces, colors),
// device workspace and the enqueueing of the HIP kernels.  No numerical
// work happens on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mrcm.h"
#include "mrcm_internal.h"

using namespace mrcm;

struct mrcm_ctx {
  int d = 0;
  int n[3] = {1, 1, 1};
  // a batch of nbatch 2-D problems on one geometry, stacked along axis 1
  // (cut cells per member; n[1] = nbatch * cut)
  int nbatch = 1, cut = 0;
  double h = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // configuration
  bool have_k = false, have_part = false;
  int S[3] = {1, 1, 1};
  int l = 0;
  int space = MRCM_SPACE_CONST;
  int beta_mode = MRCM_BETA_ALPHA;
  double beta_mbf = 1.0, beta_sm = 1.0;
  int prec = MRCM_FP64;
  int iface_solver = MRCM_IFACE_AUTO;
  double tol = 1e-12;
  int max_refine = 20;
  int bc_type[6] = {0, 0, 0, 0, 0, 0};
  int state = 0;  // 0 configured, 1 basis built, 2 solution available
  bool plan_valid = false;

  // inputs (device)
  double* logk = nullptr;  // log K: N values, or d x N (diagonal tensor, component-major)
  int kcomp = 1;           // permeability entries per cell
  double* K = nullptr;
  double* f = nullptr;
  bool have_f = false;
  double* bcv = nullptr;
  int bc_off[6] = {0, 0, 0, 0, 0, 0};
  int nbcv = 0;

  // plan
  Geo geo{};
  std::vector<Box> obox, pbox;
  std::vector<Seed> seeds, basis;
  std::vector<int> seed_off;
  std::vector<Iface> ifc;
  std::vector<int> members;
  int member_off[9] = {0};
  int nX = 0, kl = 0, ku = 0, ldab = 0;
  int mom_rows = 0;  // largest number of equation rows of one interface
  long long fac_n = 0, facp_n = 0, scr_n = 0, scro_n = 0, scrp_n = 0;

  // device plan
  Box* d_obox = nullptr;
  Box* d_pbox = nullptr;
  Seed* d_seeds = nullptr;
  Seed* d_basis = nullptr;
  int* d_seed_off = nullptr;
  Iface* d_ifc = nullptr;
  int* d_members = nullptr;
  Box* d_obox_col = nullptr;  // oversampled boxes in colour order (members order)

  // device workspace
  double *fac = nullptr, *facs = nullptr, *facp = nullptr, *scr = nullptr;
  double* fact = nullptr;  // twisted-sweep factors (backward inverses, meeting block), fac layout
  // Algorithm 1, Step 6: factors of the oversampled boxes with the smoothing
  // Robin parameter when it differs from the basis one (facs / facts, or
  // fac32s in the FP32 form), built by mrcm_build_basis
  double* facts = nullptr;
  float* fac32s = nullptr;
  size_t lds_factor = 0;
  double *tco = nullptr, *tcp = nullptr;  // block couplings of the boxes / subdomains
  bool wave = false;                      // 2-D boxes with blocks of <= 32 cells
  bool d3 = false;                        // 3-D boxes with plane blocks of <= 64 cells
  size_t lds3_basis = 0, lds3_part = 0, lds3_smooth = 0;
  // the same in the FP32 form (local3f.hip)
  size_t lds3f_basis = 0, lds3f_part = 0, lds3f_smooth = 0;
  int nw3_box = 4, nw3_part = 4;  // wavefronts per 3-D box (oversampled, subdomain)
  size_t lds_basis = 0, lds_part = 0, lds_smooth = 0;
  size_t lds32_basis = 0, lds32_part = 0, lds32_smooth = 0;
  float *fac32 = nullptr, *facp32 = nullptr;
  int* d_iters = nullptr;
  unsigned long long* d_resid = nullptr;
  double *Pk = nullptr, *tr_u = nullptr, *tr_phi = nullptr, *tr_beta = nullptr;
  double *pbar = nullptr, *ubar = nullptr, *pibar = nullptr;
  double *AB = nullptr, *rhs = nullptr, *X = nullptr;
  double *p = nullptr, *gflux = nullptr, *partial = nullptr;
  int* flags = nullptr;
  int* flags_host = nullptr;  // pinned copy target of the error flags
  double* stage_host = nullptr;  // pinned copy target of small results (16 doubles)
  bool flags_zero = false;    // flags cleared by the last check, no work since

  // conservation and continuity measures (balance.hip): partial sums,
  // results, the largest relative interface jumps after the last
  // mrcm_solve_interface (its residual check) and after mrcm_get_balance,
  // output copies for mrcm_rel_error
  double *bal_partial = nullptr, *bal_out = nullptr;
  unsigned long long *jmax_solve = nullptr, *jmax_bal = nullptr;
  double *cmp_p = nullptr, *cmp_f = nullptr;
  double iface_check_tol = 1e-5;

  // block cyclic reduction of the interface system over the layers of
  // subdomains along the last axis (bcr.hip)
  struct BcrOp {
    int kind;  // 0 inverses, 1 block products, 2 block-vector products,
               // 3 independent products (off, cnt) and vector products (off2, cnt2)
    int off, cnt;
    int n, ld;  // operand size and leading dimension (kinds 0, 1, 3)
    int off2 = 0, cnt2 = 0;
  };
  bool use_bcr = false;
  // two-level solver (iface_lsc.cpp) for 3-D grids whose layers exceed the
  // cyclic reduction's block
  Lsc* lsc = nullptr;
  bool use_lsc = false;
  int bcr_M = 0, bcr_bp = 0;
  std::vector<BcrOp> bcr_ops;
  int *d_row_lvl = nullptr, *d_row_loc = nullptr, *d_col_lvl = nullptr, *d_col_loc = nullptr;
  int* d_lsize = nullptr;
  long long* d_binv = nullptr;
  int* d_binvn = nullptr;  // pivots each inverse needs (its layer's size, rounded up to 4)
  BcrGemm* d_bgemm = nullptr;
  BcrGemv* d_bgemv = nullptr;
  double *bpool = nullptr, *bvec = nullptr;

  // smoothing execution: threads per box (0 = autotune on first use), the
  // chosen value, and the captured sweep graph
  int smooth_nt_req = 0, smooth_nt = 0;
  // 3-D FP32 smoothing: planes whose inverses a box holds in registers
  // across its refinement sweeps (8, 4, 2 or 0), chosen by the autotuner
  int smooth_cached = 8;
  bool use_graph = true;
  // one cooperative launch per mrcm_smooth call (FP64 wave kernels), with
  // at most persist_groups workgroups (0 = as many as fit)
  bool persist = false, persist_used = false;
  int persist_groups = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_steps = 0;  // smoothing steps the captured graph holds
  // phase timing: events recorded around the phases of each call (the
  // ms_* fields of mrcm_stats); off, the calls enqueue kernels only
  bool timing = true;
  bool deferred = false;      // error flags read by mrcm_wait only
  double* p_tune = nullptr;
  double* gflux_tune = nullptr;
  double ms_autotune = 0.0;

  // reverse mode: checkpoints of the smoothing state and adjoint workspace
  bool ckpt = false;
  // error flags: work that can set them bumps epoch; check_flags reads the
  // flags once per epoch (later output calls add no flag-setting work)
  long long epoch = 0, checked_epoch = -1;
  double *ck_p = nullptr, *ck_g = nullptr;
  int ck_cap = 0, n_ck = 0, n_phase = 0;
  double *a_pb = nullptr, *a_gfb = nullptr, *a_Kb = nullptr, *a_Xb = nullptr, *a_nu = nullptr;
  double *a_trub = nullptr, *a_trphib = nullptr, *a_trbetab = nullptr, *a_ubarb = nullptr;
  double *a_pibarb = nullptr, *a_mean = nullptr;
  int* d_seed_sub = nullptr;
  size_t lds_adj_smooth = 0, lds_adj_basis = 0, lds_adj_part = 0;
  size_t lds_adj32_smooth = 0, lds_adj32_basis = 0, lds_adj32_part = 0;

  hipEvent_t ev[12] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  bool timed_basis = false, timed_iface = false, timed_smooth = false;
  int n_local_solves = 0;
  int n_smooth_launches = 0;
  int n_smooth_phases = 0;
};

namespace {

mrcm_status fail(mrcm_ctx* c, mrcm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

#define HIPCHK(ctx, call)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(ctx, e_ == hipErrorOutOfMemory ? MRCM_ENOMEM : MRCM_EDEVICE, "%s: %s", \
                  #call, hipGetErrorString(e_));                                          \
  } while (0)

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void drop_graph(mrcm_ctx* c);

// MRCM_IFACE_AUTO takes the pivoted banded LU instead of the cyclic
// reduction (which does not pivot) for basis Robin parameters alpha above
// 1e4: measured on the device, the reduction's componentwise backward error
// grows from 1e-15 at alpha = 1 to 1e-9 at 1e4 and breaks down (5e-3 to 1)
// from 1e6 on, where the banded LU stays below 1e-6.
bool auto_prefers_lu(const mrcm_ctx* c) {
  return c->beta_mode == MRCM_BETA_ALPHA && c->beta_mbf > 1e4;
}

void free_plan(mrcm_ctx* c) {
  dfree(c->d_obox); dfree(c->d_pbox); dfree(c->d_seeds); dfree(c->d_basis);
  dfree(c->d_seed_off); dfree(c->d_ifc); dfree(c->d_members); dfree(c->d_obox_col);
  dfree(c->fac); dfree(c->fact); dfree(c->facs); dfree(c->facts); dfree(c->fac32s); dfree(c->facp); dfree(c->scr); dfree(c->tco); dfree(c->tcp);
  dfree(c->fac32); dfree(c->facp32); dfree(c->d_iters); dfree(c->d_resid);
  dfree(c->Pk); dfree(c->tr_u); dfree(c->tr_phi); dfree(c->tr_beta);
  dfree(c->pbar); dfree(c->ubar); dfree(c->pibar);
  dfree(c->AB); dfree(c->rhs); dfree(c->X); dfree(c->p); dfree(c->gflux); dfree(c->partial);
  dfree(c->d_row_lvl); dfree(c->d_row_loc); dfree(c->d_col_lvl); dfree(c->d_col_loc);
  dfree(c->d_lsize); dfree(c->d_binv); dfree(c->d_binvn); dfree(c->d_bgemm); dfree(c->d_bgemv);
  dfree(c->bpool); dfree(c->bvec);
  dfree(c->p_tune); dfree(c->gflux_tune);
  dfree(c->ck_p); dfree(c->ck_g);
  c->ck_cap = c->n_ck = c->n_phase = 0;
  dfree(c->a_pb); dfree(c->a_gfb); dfree(c->a_Kb); dfree(c->a_Xb); dfree(c->a_nu);
  dfree(c->a_trub); dfree(c->a_trphib); dfree(c->a_trbetab); dfree(c->a_ubarb);
  dfree(c->a_pibarb); dfree(c->a_mean); dfree(c->d_seed_sub);
  dfree(c->bal_partial); dfree(c->bal_out); dfree(c->jmax_solve); dfree(c->jmax_bal);
  dfree(c->cmp_p); dfree(c->cmp_f);
  drop_graph(c);
  c->smooth_nt = 0;
  lsc_destroy(c->lsc);
  c->lsc = nullptr;
  c->use_lsc = false;
  c->use_bcr = false;
  c->bcr_ops.clear();
  c->plan_valid = false;
}

int side_faces(const mrcm_ctx* c, const int lo[3], const int hi[3], int a) {
  int nf = 1;
  for (int b = 0; b < c->d; ++b)
    if (b != a) nf *= hi[b] - lo[b];
  return nf;
}

void sub_coords(const mrcm_ctx* c, int i, int ic[3]) {
  int r = i;
  for (int a = 0; a < 3; ++a) {
    const int Ma = a < c->d ? c->geo.M[a] : 1;
    ic[a] = r % Ma;
    r /= Ma;
  }
}

int neighbor(const mrcm_ctx* c, int i, int q) {
  const int a = q >> 1, s = q & 1;
  int ic[3];
  sub_coords(c, i, ic);
  const int t = ic[a] + (s ? 1 : -1);
  if (off_subgrid(c->geo, a, ic[a], t)) return -1;
  int stride = 1;
  for (int b = 0; b < a; ++b) stride *= c->geo.M[b];
  return i + (s ? stride : -stride);
}

// Seed family on side q of box [lo, hi) (window = Omega_i for FINE).
void family(const mrcm_ctx* c, int q, const int lo[3], const int hi[3], const int wlo[3],
            const int whi[3], std::vector<Seed>& out) {
  const int a = q >> 1;
  if (c->space == MRCM_SPACE_CONST) {
    out.push_back(Seed{q, 0, 0, 0});
  } else if (c->space == MRCM_SPACE_LINEAR) {
    out.push_back(Seed{q, 0, 0, 0});
    for (int b = 0; b < c->d; ++b)
      if (b != a) out.push_back(Seed{q, 1, b, 0});
  } else {
    // faces of the side whose tangential position lies inside the window
    const int nf = side_faces(c, lo, hi, a);
    for (int f = 0; f < nf; ++f) {
      int r = f;
      bool keep = true;
      for (int b = 0; b < c->d; ++b) {
        if (b == a) continue;
        const int m = hi[b] - lo[b];
        const int x = lo[b] + r % m;
        r /= m;
        if (x < wlo[b] || x >= whi[b]) keep = false;
      }
      if (keep) out.push_back(Seed{q, 2, 0, f});
    }
  }
}

// Plan of the block cyclic reduction (bcr.hip).  Equations are assigned to
// subdomains: the flux rows of Gamma_ij to the lower index i, the pressure
// rows to the higher index j; within a subdomain they follow its Gamma sides
// in side order, which pairs them with the seeds of the same side.  A layer
// is the set of subdomains with the same last-axis coordinate; the system is
// block tridiagonal over layers.  Returns false (band LU is used) when a
// layer block is not square or exceeds kBcrMaxBlock.
bool bcr_plan(mrcm_ctx* c, std::vector<int>& row_lvl, std::vector<int>& row_loc,
              std::vector<int>& col_lvl, std::vector<int>& col_loc, std::vector<int>& lsize,
              std::vector<long long>& inv, std::vector<int>& invn,
              std::vector<BcrGemm>& gemm, std::vector<BcrGemv>& gemv) {
  const Geo& g = c->geo;
  const int d = c->d, nsub = g.nsub, n = c->nX;
  const int M = g.M[d - 1];
  const int P = nsub / M;  // subdomains per layer (contiguous indices)
  std::vector<int> ifc_of(3 * nsub, -1);
  for (size_t k = 0; k < c->ifc.size(); ++k) ifc_of[3 * c->ifc[k].i + c->ifc[k].axis] = (int)k;
  row_lvl.assign(n, -1);
  row_loc.assign(n, -1);
  col_lvl.assign(n, -1);
  col_loc.assign(n, -1);
  std::vector<int> rows(M, 0), cols(M, 0);
  for (int i = 0; i < nsub; ++i) {
    const int k = i / P;
    for (int cc = c->seed_off[i]; cc < c->seed_off[i + 1]; ++cc) {
      col_lvl[cc] = k;
      col_loc[cc] = cols[k]++;
    }
    for (int q = 0; q < 2 * d; ++q) {
      const int j = neighbor(c, i, q);
      if (j < 0) continue;
      const int a = q >> 1;
      const bool lower = q & 1;  // i is the lower index of the interface
      const int f = ifc_of[3 * (lower ? i : j) + a];
      if (f < 0) return false;
      const Iface& F = c->ifc[f];
      const int r0 = F.row0 + (lower ? 0 : F.nbasis);
      for (int mu = 0; mu < F.nbasis; ++mu) {
        row_lvl[r0 + mu] = k;
        row_loc[r0 + mu] = rows[k]++;
      }
    }
  }
  int bp = 0;
  for (int k = 0; k < M; ++k) {
    if (rows[k] != cols[k]) return false;
    bp = std::max(bp, rows[k]);
  }
  for (int r = 0; r < n; ++r)
    if (row_lvl[r] < 0) return false;
  // tile of the block products; above kBcrInvMax the inverse works on
  // halves, which must be tiles too
  bp = bp <= kBcrInvMax ? (bp + 31) / 32 * 32 : (bp + 63) / 64 * 64;
  if (bp == 0 || bp > kBcrMaxBlock) return false;
  lsize = rows;
  c->bcr_M = M;
  c->bcr_bp = bp;

  // schedule; block slots: D_k = k, L_k = M+k, U_k = 2M+k, then F_k = 3M+k,
  // G_k = 4M+k for the layers eliminated at some level; vectors: r_k = k,
  // g_k = M+k, x_k = 2M+k.  A reduced L_j / U_j is written to the slot of
  // the eliminated neighbour's L / U, which is no longer read.
  std::vector<int> dsl(M), lsl(M), usl(M);
  for (int k = 0; k < M; ++k) {
    dsl[k] = k;
    lsl[k] = M + k;
    usl[k] = 2 * M + k;
  }
  auto F = [&](int k) { return 3 * M + k; };
  auto G = [&](int k) { return 4 * M + k; };
  auto rv = [&](int k) { return k; };
  auto gv = [&](int k) { return M + k; };
  auto xv = [&](int k) { return 2 * M + k; };
  const long long bs = (long long)bp * bp;
  auto op = [&](int kind, int off, int cnt, int nn = 0, int ld = 0) {
    if (cnt > 0) c->bcr_ops.push_back(mrcm_ctx::BcrOp{kind, off, cnt, nn, ld});
  };
  // products and vector products that read nothing the other writes
  auto op_pair = [&](int goff, int gcnt, int voff, int vcnt) {
    if (gcnt == 0) return op(2, voff, vcnt);
    if (vcnt == 0) return op(1, goff, gcnt, bp, bp);
    mrcm_ctx::BcrOp o{3, goff, gcnt, bp, bp};
    o.off2 = voff;
    o.cnt2 = vcnt;
    c->bcr_ops.push_back(o);
  };
  // a product task on whole blocks (slots < 0 drop a term)
  auto GM = [&](int cs, int c0, int a1, int b1, int a2, int b2, double al1, double al2) {
    auto o = [&](int slot) { return slot < 0 ? -1LL : slot * bs; };
    return BcrGemm{o(cs), o(c0), o(a1), o(b1), o(a2), o(b2), al1, al2};
  };
  // In-place inverses of the blocks in slots `blk`.  Up to kBcrInvMax one
  // Gauss-Jordan workgroup per block; above, the two-by-two form
  //   [A B; C D]^-1 = [A' - B' T2, B'; C', S^-1],  A' = A^-1, T1 = A' B,
  //   T2 = C A', S = D - C T1, B' = -T1 S^-1, C' = -S^-1 T2,
  // with T1 and T2 in the scratch slots s1 and s2 (quarters, ld = bp).
  auto inverses = [&](const std::vector<int>& blk, const std::vector<int>& s1,
                      const std::vector<int>& s2) {
    const int nb = (int)blk.size();
    if (nb == 0) return;
    // pivots a block's inverse needs: its layer's size rounded up to the
    // four pivots of a step (the padding beyond is identity, which a pivot
    // step leaves unchanged)
    auto piv = [](int nn) { return nn <= 0 ? 0 : (nn + 3) / 4 * 4; };
    if (bp <= kBcrInvMax) {
      const int o = (int)inv.size();
      for (int b : blk) {
        inv.push_back(b * bs);
        invn.push_back(std::min(piv(lsize[b]), bp));
      }
      op(0, o, nb, bp, bp);
      return;
    }
    const int hh = bp / 2;
    auto A = [&](int i) { return blk[i] * bs; };
    auto B = [&](int i) { return blk[i] * bs + hh; };
    auto C = [&](int i) { return blk[i] * bs + (long long)hh * bp; };
    auto D = [&](int i) { return blk[i] * bs + (long long)hh * bp + hh; };
    auto T1 = [&](int i) { return s1[i] * bs; };
    auto T2 = [&](int i) { return s2[i] * bs; };
    int o = (int)inv.size();
    for (int i = 0; i < nb; ++i) {
      inv.push_back(A(i));
      invn.push_back(std::min(piv(lsize[blk[i]]), hh));
    }
    op(0, o, nb, hh, bp);
    o = (int)gemm.size();
    for (int i = 0; i < nb; ++i) {
      gemm.push_back(BcrGemm{T1(i), -1, A(i), B(i), -1, -1, 1.0, 0.0});
      gemm.push_back(BcrGemm{T2(i), -1, C(i), A(i), -1, -1, 1.0, 0.0});
    }
    op(1, o, 2 * nb, hh, bp);
    o = (int)gemm.size();
    for (int i = 0; i < nb; ++i) gemm.push_back(BcrGemm{D(i), D(i), C(i), T1(i), -1, -1, -1.0, 0.0});
    op(1, o, nb, hh, bp);
    o = (int)inv.size();
    for (int i = 0; i < nb; ++i) {
      inv.push_back(D(i));
      invn.push_back(std::min(piv(lsize[blk[i]] - hh), hh));
    }
    op(0, o, nb, hh, bp);
    o = (int)gemm.size();
    for (int i = 0; i < nb; ++i) {
      gemm.push_back(BcrGemm{B(i), -1, T1(i), D(i), -1, -1, -1.0, 0.0});
      gemm.push_back(BcrGemm{C(i), -1, D(i), T2(i), -1, -1, -1.0, 0.0});
    }
    op(1, o, 2 * nb, hh, bp);
    o = (int)gemm.size();
    for (int i = 0; i < nb; ++i) gemm.push_back(BcrGemm{A(i), A(i), B(i), T2(i), -1, -1, -1.0, 0.0});
    op(1, o, nb, hh, bp);
  };
  std::vector<std::vector<BcrGemv>> back;
  std::vector<int> idx(M);
  for (int k = 0; k < M; ++k) idx[k] = k;
  c->bcr_ops.clear();
  while (idx.size() > 1) {
    const int L = (int)idx.size();
    // eliminated layers (odd positions): E_k = D_k^{-1}, F_k, G_k, g_k
    // (the F and G slots of k are free until then: scratch of the inverse)
    {
      std::vector<int> blk, s1, s2;
      for (int t = 1; t < L; t += 2) {
        blk.push_back(dsl[idx[t]]);
        s1.push_back(F(idx[t]));
        s2.push_back(G(idx[t]));
      }
      inverses(blk, s1, s2);
    }
    // F_k = E_k L_k, G_k = E_k U_k and g_k = E_k r_k read only E, L, U, r:
    // one launch
    int o = (int)gemm.size();
    for (int t = 1; t < L; t += 2) {
      const int k = idx[t];
      gemm.push_back(GM(F(k), -1, dsl[k], lsl[k], -1, -1, 1.0, 0.0));
      if (t + 1 < L) gemm.push_back(GM(G(k), -1, dsl[k], usl[k], -1, -1, 1.0, 0.0));
    }
    const int ov0 = (int)gemv.size();
    for (int t = 1; t < L; t += 2) {
      const int k = idx[t];
      gemv.push_back(BcrGemv{gv(k), -1, dsl[k], rv(k), -1, -1, 1.0, 0.0});
    }
    op_pair(o, (int)gemm.size() - o, ov0, (int)gemv.size() - ov0);
    // kept layers (even positions)
    std::vector<int> nl(M, -1), nu(M, -1);
    o = (int)gemm.size();
    const int ov = (int)gemv.size();
    for (int t = 0; t < L; t += 2) {
      const int j = idx[t];
      const bool hl = t > 0, hr = t + 1 < L;
      const int km = hl ? idx[t - 1] : -1, kp = hr ? idx[t + 1] : -1;
      BcrGemm Dt = GM(dsl[j], dsl[j], -1, -1, -1, -1, -1.0, -1.0);
      BcrGemv Rt{rv(j), rv(j), -1, -1, -1, -1, -1.0, -1.0};
      if (hl) {
        Dt.a1 = lsl[j] * bs;
        Dt.b1 = G(km) * bs;
        Rt.a1 = lsl[j];
        Rt.x1 = gv(km);
      }
      if (hr) {
        (hl ? Dt.a2 : Dt.a1) = usl[j] * bs;
        (hl ? Dt.b2 : Dt.b1) = F(kp) * bs;
        (hl ? Rt.a2 : Rt.a1) = usl[j];
        (hl ? Rt.x2 : Rt.x1) = gv(kp);
      }
      gemm.push_back(Dt);
      gemv.push_back(Rt);
      if (hl && t - 1 > 0) {
        gemm.push_back(GM(lsl[km], -1, lsl[j], F(km), -1, -1, -1.0, 0.0));
        nl[j] = lsl[km];
      }
      if (hr && t + 2 < L) {
        gemm.push_back(GM(usl[kp], -1, usl[j], G(kp), -1, -1, -1.0, 0.0));
        nu[j] = usl[kp];
      }
    }
    // the kept-layer products write D_j and the eliminated neighbours' L/U
    // slots; the vector products read L_j, U_j (kept slots) and g: one launch
    op_pair(o, (int)gemm.size() - o, ov, (int)gemv.size() - ov);
    // back substitution of this level, replayed in reverse order
    std::vector<BcrGemv> bk;
    for (int t = 1; t < L; t += 2) {
      const int k = idx[t];
      BcrGemv B{xv(k), gv(k), F(k), xv(idx[t - 1]), -1, -1, -1.0, -1.0};
      if (t + 1 < L) {
        B.a2 = G(k);
        B.x2 = xv(idx[t + 1]);
      }
      bk.push_back(B);
    }
    back.push_back(bk);
    std::vector<int> keep;
    for (int t = 0; t < L; t += 2) {
      const int j = idx[t];
      lsl[j] = nl[j];
      usl[j] = nu[j];
      keep.push_back(j);
    }
    idx.swap(keep);
  }
  const int k0 = idx[0];
  inverses({dsl[k0]}, {F(k0)}, {G(k0)});
  int o = (int)gemv.size();
  gemv.push_back(BcrGemv{xv(k0), -1, dsl[k0], rv(k0), -1, -1, 1.0, 0.0});
  op(2, o, 1);
  for (int lv = (int)back.size() - 1; lv >= 0; --lv) {
    o = (int)gemv.size();
    for (const auto& B : back[lv]) gemv.push_back(B);
    op(2, o, (int)back[lv].size());
  }
  return true;
}

mrcm_status make_plan(mrcm_ctx* c) {
  free_plan(c);
  Geo& g = c->geo;
  g = Geo{};
  g.d = c->d;
  g.l = c->l;
  g.h = c->h;
  g.area = std::pow(c->h, c->d - 1);
  g.vol = std::pow(c->h, c->d);
  g.beta_mode = c->beta_mode == MRCM_BETA_CONST ? 1 : 0;
  g.kc = c->kcomp;
  g.ncells = 1;
  g.nsub = 1;
  g.neumann = 1;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = a < c->d ? c->n[a] : 1;
    g.S[a] = a < c->d ? c->S[a] : 1;
    g.M[a] = g.n[a] / g.S[a];
    g.ncells *= g.n[a];
    g.nsub *= g.M[a];
  }
  for (int q = 0; q < 6; ++q) {
    g.bc_type[q] = c->bc_type[q];
    g.bc_off[q] = c->bc_off[q];
    if (q < 2 * c->d && c->bc_type[q]) g.neumann = 0;
  }
  int off = 0;
  for (int q = 0; q < 6; ++q) {
    g.gside_off[q] = off;
    if (q < 2 * c->d) {
      int nf = 1;
      for (int b = 0; b < c->d; ++b)
        if (b != (q >> 1)) nf *= g.S[b];
      off += nf;
    }
  }
  g.gstride = off;
  g.nfaceg = 0;
  g.cut = c->cut;
  g.mcut = c->cut > 0 ? c->cut / g.S[1] : 0;
  if (c->nbatch > 1 && g.neumann)
    return fail(c, MRCM_EINVAL, "a batch needs a pressure (Dirichlet) boundary: each member would need its own gauge");

  const int nsub = g.nsub;
  c->seeds.clear();
  c->seed_off.assign(nsub + 1, 0);
  c->obox.resize(nsub);
  c->pbox.resize(nsub);
  long long fac = 0, facp = 0, scr = 0, scrp = 0;
  for (int i = 0; i < nsub; ++i) {
    int ic[3];
    sub_coords(c, i, ic);
    int wlo[3], whi[3], lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      wlo[a] = ic[a] * g.S[a];
      whi[a] = wlo[a] + g.S[a];
      lo[a] = a < c->d ? std::max(wlo[a] - c->l, 0) : 0;
      hi[a] = a < c->d ? std::min(whi[a] + c->l, g.n[a]) : 1;
    }
    if (g.cut > 0) {
      // a batch member's boxes end at its cuts, as at the domain boundary
      const int m0 = wlo[1] / g.cut * g.cut;
      lo[1] = std::max(lo[1], m0);
      hi[1] = std::min(hi[1], m0 + g.cut);
    }
    c->seed_off[i] = (int)c->seeds.size();
    for (int q = 0; q < 2 * c->d; ++q)
      if (neighbor(c, i, q) >= 0) family(c, q, lo, hi, wlo, whi, c->seeds);
    Box& B = c->obox[i];
    B = Box{};
    for (int a = 0; a < 3; ++a) { B.lo[a] = lo[a]; B.hi[a] = hi[a]; }
    B.sub = i;
    B.nb = 1;
    for (int a = 0; a < c->d - 1; ++a) B.nb *= hi[a] - lo[a];
    B.nblk = hi[c->d - 1] - lo[c->d - 1];
    B.ncell = B.nb * B.nblk;
    B.seed0 = c->seed_off[i];
    B.nrhs = (int)c->seeds.size() - B.seed0;
    B.fac = fac;
    fac += (long long)B.nblk * B.nb * B.nb;
    B.scr = scr;
    scr += (long long)B.ncell * std::max(B.nrhs, 1);
    if (B.nb > kMaxBlock)
      return fail(c, MRCM_EINVAL, "oversampled box block of %d cells exceeds %d", B.nb, kMaxBlock);
    if (B.nrhs > kMaxRhs)
      return fail(c, MRCM_EINVAL, "%d seeds on one box exceed %d", B.nrhs, kMaxRhs);
    Box& P = c->pbox[i];
    P = Box{};
    for (int a = 0; a < 3; ++a) { P.lo[a] = wlo[a]; P.hi[a] = whi[a]; }
    P.sub = i;
    P.nb = 1;
    for (int a = 0; a < c->d - 1; ++a) P.nb *= whi[a] - wlo[a];
    P.nblk = whi[c->d - 1] - wlo[c->d - 1];
    P.ncell = P.nb * P.nblk;
    P.nrhs = 1;
    P.fac = facp;
    facp += (long long)P.nblk * P.nb * P.nb;
    P.scr = scrp;
    scrp += P.ncell;
    if (P.nb > kMaxBlock)
      return fail(c, MRCM_EINVAL, "subdomain block of %d cells exceeds %d", P.nb, kMaxBlock);
  }
  c->seed_off[nsub] = (int)c->seeds.size();
  c->nX = c->seed_off[nsub];
  c->fac_n = fac;
  c->facp_n = facp;
  c->scr_n = std::max(scr, scrp);
  c->scro_n = scr;
  c->scrp_n = scrp;
  c->wave = c->d == 2;
  c->lds_basis = c->lds_part = c->lds_smooth = c->lds_factor = 0;
  c->lds_adj_smooth = c->lds_adj_basis = c->lds_adj_part = 0;
  c->lds_adj32_smooth = c->lds_adj32_basis = c->lds_adj32_part = 0;
  for (int i = 0; i < nsub; ++i) {
    const Box& B = c->obox[i];
    const Box& P = c->pbox[i];
    if (B.nb > 32 || P.nb > 32) c->wave = false;
    const int bm0 = B.hi[0] - B.lo[0], bm1 = B.hi[1] - B.lo[1];
    const int kc = c->kcomp;
    c->lds_basis = std::max(c->lds_basis, wave_basis_lds_bytes(bm0, bm1, std::max(B.nrhs, 1), kc));
    c->lds_factor = std::max(c->lds_factor, wave_basis_lds_bytes(bm0, bm1, 0, kc));
    c->lds_smooth = std::max(c->lds_smooth, wave_smooth_lds_bytes(bm0, bm1, kc));
    c->lds_part = std::max(c->lds_part, wave_lds_bytes(P.hi[0] - P.lo[0], P.hi[1] - P.lo[1], 1, kc));
    c->lds32_basis = std::max(c->lds32_basis, wave32_lds_bytes(bm0, bm1, std::max(B.nrhs, 1), 0, kc));
    c->lds32_smooth = std::max(c->lds32_smooth, wave32_smooth_lds_bytes(bm0, bm1, kc));
    c->lds32_part = std::max(c->lds32_part, wave32_lds_bytes(P.hi[0] - P.lo[0], P.hi[1] - P.lo[1], 1, 1, kc));
    if (c->d == 2) {
      for (int f32 = 0; f32 < 2; ++f32) {
        size_t& ls = f32 ? c->lds_adj32_smooth : c->lds_adj_smooth;
        size_t& lb = f32 ? c->lds_adj32_basis : c->lds_adj_basis;
        size_t& lp = f32 ? c->lds_adj32_part : c->lds_adj_part;
        ls = std::max(ls, adj_smooth_lds_bytes(bm0, bm1, f32));
        lb = std::max(lb, adj_basis_lds_bytes(bm0, bm1, std::max(B.nrhs, 1), f32));
        lp = std::max(lp, adj_part_lds_bytes(P.hi[0] - P.lo[0], P.hi[1] - P.lo[1], f32));
      }
    }
  }
  if (c->lds_basis > 150 * 1024 || c->lds_smooth > 150 * 1024 || 2 * c->lds_part + 16 > 150 * 1024)
    c->wave = false;
  // 3-D boxes: one wave per box with plane blocks of at most 64 cells
  c->d3 = c->d == 3;
  c->lds3_basis = c->lds3_part = c->lds3_smooth = 0;
  c->lds3f_basis = c->lds3f_part = c->lds3f_smooth = 0;
  int nb3_box = 1, nb3_part = 1;
  for (int i = 0; i < nsub && c->d3; ++i) {
    const Box& B = c->obox[i];
    const Box& P = c->pbox[i];
    if (B.nb > 64 || P.nb > 64) c->d3 = false;
    nb3_box = std::max(nb3_box, B.nb);
    nb3_part = std::max(nb3_part, P.nb);
    const int m[3] = {B.hi[0] - B.lo[0], B.hi[1] - B.lo[1], B.hi[2] - B.lo[2]};
    const int kc = c->kcomp;
    c->lds3_basis = std::max(c->lds3_basis, box3_lds_bytes(m[0], m[1], m[2], std::max(B.nrhs, 1), kc));
    c->lds3_smooth = std::max(c->lds3_smooth, box3_lds_bytes(m[0], m[1], m[2], 1, kc));
    c->lds3_part = std::max(c->lds3_part, box3_lds_bytes(P.hi[0] - P.lo[0], P.hi[1] - P.lo[1],
                                                         P.hi[2] - P.lo[2], 1, kc));
    c->lds3f_basis = std::max(c->lds3f_basis, box3f_lds_bytes(m[0], m[1], m[2],
                                                              std::min(std::max(B.nrhs, 1), kSeedBatch3f), 0, kc));
    c->lds3f_smooth = std::max(c->lds3f_smooth, box3f_lds_bytes(m[0], m[1], m[2], 1, 1, kc));
    c->lds3f_part = std::max(c->lds3f_part, box3f_lds_bytes(P.hi[0] - P.lo[0], P.hi[1] - P.lo[1],
                                                            P.hi[2] - P.lo[2], 1, 1, kc));
  }
  if (c->lds3_basis > 150 * 1024 || c->lds3_smooth > 150 * 1024 || c->lds3_part > 150 * 1024)
    c->d3 = false;
  c->nw3_box = box3_waves(nb3_box);
  c->nw3_part = box3_waves(nb3_part);

  // interfaces and their test functions
  c->ifc.clear();
  c->basis.clear();
  int row = 0;
  c->kl = 0;
  c->ku = 0;
  c->mom_rows = 0;
  for (int i = 0; i < nsub; ++i) {
    for (int a = 0; a < c->d; ++a) {
      const int j = neighbor(c, i, 2 * a + 1);
      if (j < 0) continue;
      int ic[3], wlo[3], whi[3];
      sub_coords(c, i, ic);
      for (int b = 0; b < 3; ++b) {
        wlo[b] = ic[b] * g.S[b];
        whi[b] = wlo[b] + g.S[b];
      }
      Iface F;
      F.i = i;
      F.j = j;
      F.axis = a;
      F.row0 = row;
      F.basis0 = (int)c->basis.size();
      family(c, 2 * a + 1, wlo, whi, wlo, whi, c->basis);
      F.nbasis = (int)c->basis.size() - F.basis0;
      c->mom_rows = std::max(c->mom_rows, 2 * F.nbasis);
      const int cmin = c->seed_off[i];
      const int cmax = c->seed_off[j + 1] - 1;
      for (int r = row; r < row + 2 * F.nbasis; ++r) {
        c->kl = std::max(c->kl, r - cmin);
        c->ku = std::max(c->ku, cmax - r);
      }
      row += 2 * F.nbasis;
      c->ifc.push_back(F);
    }
  }
  if (row != c->nX)
    return fail(c, MRCM_EINVAL,
                "interface system not square (Proposition 1): %d equations, %d unknowns", row,
                c->nX);
  c->ldab = c->kl + c->ku + 1;  // row-band width (input rows, then U rows)

  // colors: parity of the subdomain index per axis
  c->members.clear();
  for (int col = 0; col < (1 << c->d); ++col) {
    c->member_off[col] = (int)c->members.size();
    for (int i = 0; i < nsub; ++i) {
      int ic[3];
      sub_coords(c, i, ic);
      int cc = 0;
      for (int a = 0; a < c->d; ++a) cc |= (ic[a] & 1) << a;
      if (cc == col) c->members.push_back(i);
    }
  }
  c->member_off[1 << c->d] = (int)c->members.size();

  // device allocations
  auto alloc = [&](auto*& ptr, size_t count) -> mrcm_status {
    using T = std::remove_reference_t<decltype(*ptr)>;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)&ptr, count * sizeof(T));
    if (e != hipSuccess) return fail(c, MRCM_ENOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
    return MRCM_OK;
  };
#define ALLOC(p, n) do { mrcm_status s_ = alloc(p, (size_t)(n)); if (s_) return s_; } while (0)
  const long long ncell_o = (long long)g.S[0] * g.S[1] * g.S[2];
  ALLOC(c->d_obox, nsub);
  ALLOC(c->d_pbox, nsub);
  ALLOC(c->d_seeds, c->seeds.size());
  ALLOC(c->d_basis, c->basis.size());
  ALLOC(c->d_seed_off, nsub + 1);
  ALLOC(c->d_ifc, c->ifc.size());
  ALLOC(c->d_members, c->members.size());
  ALLOC(c->d_obox_col, c->members.size());
  ALLOC(c->fac, c->fac_n);
  ALLOC(c->fact, c->fac_n);
  ALLOC(c->facp, c->facp_n);
  ALLOC(c->scr, c->scr_n);
  ALLOC(c->tco, c->scro_n);
  ALLOC(c->tcp, c->scrp_n);
  ALLOC(c->fac32, c->fac_n);
  ALLOC(c->facp32, c->facp_n);
  ALLOC(c->d_iters, 1);
  ALLOC(c->d_resid, 1);
  ALLOC(c->Pk, (long long)c->nX * ncell_o);
  ALLOC(c->tr_u, (long long)c->nX * g.gstride);
  ALLOC(c->tr_phi, (long long)c->nX * g.gstride);
  ALLOC(c->tr_beta, (long long)nsub * g.gstride);
  ALLOC(c->pbar, (long long)nsub * ncell_o);
  ALLOC(c->ubar, (long long)nsub * g.gstride);
  ALLOC(c->pibar, (long long)nsub * g.gstride);
  ALLOC(c->AB, 2LL * c->ldab * std::max(c->nX, 1));
  ALLOC(c->rhs, c->nX);
  ALLOC(c->X, c->nX);
  ALLOC(c->p, g.ncells);
  ALLOC(c->gflux, (long long)nsub * g.gstride);
  ALLOC(c->partial, 64);
  ALLOC(c->bal_partial, (long long)std::max(cell_balance_blocks(g), 256) * std::max(kBalParts, 2));
  ALLOC(c->bal_out, 16);
  ALLOC(c->jmax_solve, 2);
  ALLOC(c->jmax_bal, 2);
  HIPCHK(c, hipMemcpy(c->d_obox, c->obox.data(), nsub * sizeof(Box), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_pbox, c->pbox.data(), nsub * sizeof(Box), hipMemcpyHostToDevice));
  if (!c->seeds.empty())
    HIPCHK(c, hipMemcpy(c->d_seeds, c->seeds.data(), c->seeds.size() * sizeof(Seed), hipMemcpyHostToDevice));
  if (!c->basis.empty())
    HIPCHK(c, hipMemcpy(c->d_basis, c->basis.data(), c->basis.size() * sizeof(Seed), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_seed_off, c->seed_off.data(), (nsub + 1) * sizeof(int), hipMemcpyHostToDevice));
  if (!c->ifc.empty())
    HIPCHK(c, hipMemcpy(c->d_ifc, c->ifc.data(), c->ifc.size() * sizeof(Iface), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_members, c->members.data(), c->members.size() * sizeof(int), hipMemcpyHostToDevice));
  {
    std::vector<Box> col(c->members.size());
    for (size_t i = 0; i < col.size(); ++i) col[i] = c->obox[c->members[i]];
    HIPCHK(c, hipMemcpy(c->d_obox_col, col.data(), col.size() * sizeof(Box), hipMemcpyHostToDevice));
  }

  // interface solver
  c->use_bcr = false;
  const bool try_bcr = c->iface_solver == MRCM_IFACE_BCR ||
                       (c->iface_solver == MRCM_IFACE_AUTO && !auto_prefers_lu(c));
  if (c->nX > 0 && try_bcr) {
    std::vector<int> rl, ro, cl, co, ls;
    std::vector<long long> inv;
    std::vector<int> invn;
    std::vector<BcrGemm> gm;
    std::vector<BcrGemv> gv;
    const bool ok = bcr_plan(c, rl, ro, cl, co, ls, inv, invn, gm, gv);
    if (!ok && c->iface_solver == MRCM_IFACE_BCR)
      return fail(c, MRCM_EINVAL,
                  "block cyclic reduction needs square layer blocks of at most %d unknowns",
                  kBcrMaxBlock);
    if (ok) {
      const int M = c->bcr_M;
      const long long bs = (long long)c->bcr_bp * c->bcr_bp;
      ALLOC(c->d_row_lvl, c->nX);
      ALLOC(c->d_row_loc, c->nX);
      ALLOC(c->d_col_lvl, c->nX);
      ALLOC(c->d_col_loc, c->nX);
      ALLOC(c->d_lsize, M);
      ALLOC(c->d_binv, inv.size());
      ALLOC(c->d_binvn, invn.size());
      ALLOC(c->d_bgemm, gm.size());
      ALLOC(c->d_bgemv, gv.size());
      ALLOC(c->bpool, 5LL * M * bs);
      ALLOC(c->bvec, 3LL * M * c->bcr_bp);
      auto up = [&](void* dst, const void* src, size_t bytes) {
        return bytes ? hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
      };
      HIPCHK(c, up(c->d_row_lvl, rl.data(), rl.size() * sizeof(int)));
      HIPCHK(c, up(c->d_row_loc, ro.data(), ro.size() * sizeof(int)));
      HIPCHK(c, up(c->d_col_lvl, cl.data(), cl.size() * sizeof(int)));
      HIPCHK(c, up(c->d_col_loc, co.data(), co.size() * sizeof(int)));
      HIPCHK(c, up(c->d_lsize, ls.data(), ls.size() * sizeof(int)));
      HIPCHK(c, up(c->d_binv, inv.data(), inv.size() * sizeof(long long)));
      HIPCHK(c, up(c->d_binvn, invn.data(), invn.size() * sizeof(int)));
      HIPCHK(c, up(c->d_bgemm, gm.data(), gm.size() * sizeof(BcrGemm)));
      HIPCHK(c, up(c->d_bgemv, gv.data(), gv.size() * sizeof(BcrGemv)));
      c->use_bcr = true;
    }
  }
  // 3-D: the two-level reduction when the cyclic reduction's layer blocks
  // are too large (or when asked for)
  const bool try_lsc = c->iface_solver == MRCM_IFACE_LAYERED ||
                       (c->iface_solver == MRCM_IFACE_AUTO && !c->use_bcr && !auto_prefers_lu(c));
  if (c->nX > 0 && c->d == 3 && try_lsc) {
    std::vector<int> per_side((size_t)nsub * 6, 0);
    for (int i = 0; i < nsub; ++i)
      for (int k = c->seed_off[i]; k < c->seed_off[i + 1]; ++k) ++per_side[(size_t)i * 6 + c->seeds[k].side];
    std::string why;
    hipError_t he = hipSuccess;
    c->lsc = lsc_create(g, c->ifc, c->seed_off, per_side, c->nX, &why, &he);
    if (!c->lsc) {
      if (he != hipSuccess)
        return fail(c, he == hipErrorOutOfMemory ? MRCM_ENOMEM : MRCM_EDEVICE, "two-level plan: %s",
                    why.c_str());
      if (c->iface_solver == MRCM_IFACE_LAYERED)
        return fail(c, MRCM_EINVAL, "two-level interface solver: %s", why.c_str());
    } else {
      c->use_lsc = true;
    }
  } else if (c->iface_solver == MRCM_IFACE_LAYERED && c->nX > 0) {
    return fail(c, MRCM_EINVAL, "the two-level interface solver needs a 3-D grid");
  }
#undef ALLOC
  c->plan_valid = true;
  return MRCM_OK;
}

mrcm_status run_bcr_ops(mrcm_ctx* c, hipStream_t s) {
  const int bp = c->bcr_bp;
  for (const auto& o : c->bcr_ops) {
    if (o.kind == 0)
      HIPCHK(c, launch_bcr_inv(c->bpool, c->d_binv + o.off, c->d_binvn + o.off, o.cnt, o.n, o.ld,
                               c->flags, s));
    else if (o.kind == 1)
      HIPCHK(c, launch_bcr_gemm(c->bpool, c->d_bgemm + o.off, o.cnt, o.n, o.ld, s));
    else if (o.kind == 2)
      HIPCHK(c, launch_bcr_gemv(c->bpool, c->bvec, c->d_bgemv + o.off, o.cnt, bp, s));
    else
      HIPCHK(c, launch_bcr_gemm_gemv(c->bpool, c->bvec, c->d_bgemm + o.off, o.cnt,
                                     c->d_bgemv + o.off2, o.cnt2, o.n, o.ld, bp, s));
  }
  return MRCM_OK;
}

mrcm_status bcr_solve(mrcm_ctx* c, hipStream_t s) {
  const int M = c->bcr_M, bp = c->bcr_bp;
  const long long bs = (long long)bp * bp;
  (void)bs;
  // blocks and right-hand sides are in place (set up and filled by
  // mrcm_solve_interface before the moments)
  {
    mrcm_status st = run_bcr_ops(c, s);
    if (st) return st;
  }
  HIPCHK(c, launch_bcr_gather(c->bvec + 2LL * M * bp, c->d_col_lvl, c->d_col_loc, c->nX, bp, c->X, s));
  return MRCM_OK;
}

// Reads and clears the device error flags after the work enqueued so far.
mrcm_status read_flags(mrcm_ctx* c) {
  // one wait: the copy into pinned memory is ordered after the work, and
  // the flags are cleared for the next solve in the same round
  HIPCHK(c, hipMemcpyAsync(c->flags_host, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemsetAsync(c->flags, 0, sizeof(int), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int fl = *c->flags_host;
  c->flags_zero = true;
  if (!fl) c->checked_epoch = c->epoch;
  if (fl & kFlagBadK) return fail(c, MRCM_EINVAL, "permeability must be finite and positive");
  if (fl & kFlagNotPD) return fail(c, MRCM_ENOTPD, "local factorisation met a non-positive pivot");
  if (fl & kFlagSingular) return fail(c, MRCM_ESINGULAR, "interface system is singular");
  if (fl & kFlagNoConv) return fail(c, MRCM_ENOCONV, "iterative refinement did not converge");
  return MRCM_OK;
}

// End of a call that may report device-side errors: with deferred errors the
// flags stay set on the device until mrcm_wait reads them.
mrcm_status check_flags(mrcm_ctx* c) {
  if (c->deferred) return MRCM_OK;
  if (c->checked_epoch == c->epoch) return MRCM_OK;
  return read_flags(c);
}

void drop_graph(mrcm_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

void invalidate(mrcm_ctx* c, bool geometry) {
  c->state = 0;
  drop_graph(c);
  if (geometry) {
    c->plan_valid = false;
    c->smooth_nt = 0;
  }
}

}  // namespace

extern "C" {

namespace {
// Boundary values per side: faces x-fastest over the other axes; on the
// y sides of a batch, member after member.
int side_values(const mrcm_ctx* c, int side) {
  int nf = 1;
  for (int b = 0; b < c->d; ++b)
    if (b != (side >> 1)) nf *= c->n[b];
  if ((side >> 1) == 1 && c->cut > 0) nf *= c->nbatch;
  return nf;
}

mrcm_status create_ctx(int dim, const int* ncell, double h, int nbatch, void* stream, mrcm_ctx** out) {
  if (!out) return MRCM_EINVAL;
  *out = nullptr;
  if (dim != 2 && dim != 3) return MRCM_EINVAL;
  if (!ncell || !(h > 0.0) || !std::isfinite(h)) return MRCM_EINVAL;
  if (nbatch < 1 || (nbatch > 1 && dim != 2)) return MRCM_EINVAL;
  long long N = nbatch;
  for (int a = 0; a < dim; ++a) {
    if (ncell[a] <= 0) return MRCM_EINVAL;
    N *= ncell[a];
  }
  if (N > (1LL << 31) - 1) return MRCM_EINVAL;
  mrcm_ctx* c = new (std::nothrow) mrcm_ctx();
  if (!c) return MRCM_ENOMEM;
  c->d = dim;
  for (int a = 0; a < dim; ++a) c->n[a] = ncell[a];
  if (nbatch > 1) {
    c->nbatch = nbatch;
    c->cut = ncell[1];
    c->n[1] = ncell[1] * nbatch;
  }
  c->h = h;
  c->stream = (hipStream_t)stream;
  int off = 0;
  for (int q = 0; q < 2 * dim; ++q) {
    c->bc_off[q] = off;
    off += side_values(c, q);
  }
  c->nbcv = off;
  // room for a diagonal tensor's d entries per cell
  hipError_t e = hipMalloc((void**)&c->logk, (size_t)dim * N * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&c->K, (size_t)dim * N * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&c->f, N * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&c->bcv, off * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&c->flags, sizeof(int));
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->flags_host, sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->stage_host, 16 * sizeof(double), hipHostMallocDefault);
  for (int k = 0; k < 12 && e == hipSuccess; ++k) e = hipEventCreate(&c->ev[k]);
  // the error flags start clear: with deferred errors no later call clears
  // them before the first mrcm_wait
  if (e == hipSuccess) e = hipMemsetAsync(c->flags, 0, sizeof(int), c->stream);
  if (e == hipSuccess) e = launch_fill(c->bcv, 0.0, off, c->stream);
  if (e == hipSuccess) e = launch_fill(c->f, 0.0, N, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    mrcm_destroy(c);
    return e == hipErrorOutOfMemory ? MRCM_ENOMEM : MRCM_EDEVICE;
  }
  c->flags_zero = true;
  *out = c;
  return MRCM_OK;
}
}  // namespace

mrcm_status mrcm_create(int dim, const int* ncell, double h, void* stream, mrcm_ctx** out) {
  return create_ctx(dim, ncell, h, 1, stream, out);
}

mrcm_status mrcm_create_batched(int dim, const int* ncell, double h, int nbatch, void* stream,
                                mrcm_ctx** out) {
  return create_ctx(dim, ncell, h, nbatch, stream, out);
}

mrcm_status mrcm_set_permeability(mrcm_ctx* c, const double* logk_dev) {
  if (!c) return MRCM_EINVAL;
  if (!logk_dev) return fail(c, MRCM_EINVAL, "logk is NULL");
  const long long N = (long long)c->n[0] * c->n[1] * c->n[2];
  HIPCHK(c, hipMemcpyAsync(c->logk, logk_dev, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->have_k = true;
  // the box layouts hold one permeability tile per entry of a cell
  invalidate(c, c->kcomp != 1);
  c->kcomp = 1;
  return MRCM_OK;
}

mrcm_status mrcm_set_permeability_diag(mrcm_ctx* c, const double* logk_dev) {
  if (!c) return MRCM_EINVAL;
  if (!logk_dev) return fail(c, MRCM_EINVAL, "logk is NULL");
  const long long N = (long long)c->n[0] * c->n[1] * c->n[2];
  HIPCHK(c, hipMemcpyAsync(c->logk, logk_dev, (size_t)c->d * N * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream));
  c->have_k = true;
  invalidate(c, c->kcomp != c->d);
  c->kcomp = c->d;
  return MRCM_OK;
}

mrcm_status mrcm_set_source(mrcm_ctx* c, const double* f_dev) {
  if (!c) return MRCM_EINVAL;
  const long long N = (long long)c->n[0] * c->n[1] * c->n[2];
  if (f_dev) {
    HIPCHK(c, hipMemcpyAsync(c->f, f_dev, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  } else {
    HIPCHK(c, launch_fill(c->f, 0.0, N, c->stream));
  }
  c->have_f = f_dev != nullptr;
  invalidate(c, false);
  return MRCM_OK;
}

mrcm_status mrcm_set_bc(mrcm_ctx* c, int side, mrcm_bc_type type, const double* val_dev) {
  if (!c) return MRCM_EINVAL;
  if (side < 0 || side >= 2 * c->d) return fail(c, MRCM_EINVAL, "side %d out of range", side);
  if (type != MRCM_BC_NEUMANN && type != MRCM_BC_DIRICHLET) return fail(c, MRCM_EINVAL, "bad bc type");
  const int nf = side_values(c, side);
  if (val_dev) {
    HIPCHK(c, hipMemcpyAsync(c->bcv + c->bc_off[side], val_dev, nf * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
  } else {
    HIPCHK(c, launch_fill(c->bcv + c->bc_off[side], 0.0, nf, c->stream));
  }
  const bool changed = c->bc_type[side] != (int)type;
  c->bc_type[side] = (int)type;
  invalidate(c, changed);
  return MRCM_OK;
}

mrcm_status mrcm_set_partition(mrcm_ctx* c, const int* sub, int overlap) {
  if (!c) return MRCM_EINVAL;
  if (!sub) return fail(c, MRCM_EINVAL, "sub is NULL");
  int smin = 1 << 30;
  for (int a = 0; a < c->d; ++a) {
    if (sub[a] <= 0 || c->n[a] % sub[a])
      return fail(c, MRCM_EINVAL, "axis %d: %d cells not a multiple of subdomain size %d", a, c->n[a], sub[a]);
    smin = std::min(smin, sub[a]);
  }
  if (overlap < 0 || overlap > smin - 1)
    return fail(c, MRCM_EINVAL, "overlap must satisfy 0 <= l <= min(sub) - 1");
  if (c->cut > 0 && c->cut % sub[1])
    return fail(c, MRCM_EINVAL, "batch member: %d cells along y not a multiple of subdomain size %d",
                c->cut, sub[1]);
  for (int a = 0; a < c->d; ++a) c->S[a] = sub[a];
  c->l = overlap;
  c->have_part = true;
  invalidate(c, true);
  return MRCM_OK;
}

mrcm_status mrcm_set_interface_solver(mrcm_ctx* c, mrcm_iface_solver solver) {
  if (!c) return MRCM_EINVAL;
  if (solver < MRCM_IFACE_AUTO || solver > MRCM_IFACE_LAYERED) return fail(c, MRCM_EINVAL, "bad interface solver");
  c->iface_solver = solver;
  invalidate(c, true);
  return MRCM_OK;
}

mrcm_status mrcm_set_interface_space(mrcm_ctx* c, mrcm_space space) {
  if (!c) return MRCM_EINVAL;
  if (space < MRCM_SPACE_CONST || space > MRCM_SPACE_FINE) return fail(c, MRCM_EINVAL, "bad space");
  c->space = space;
  invalidate(c, true);
  return MRCM_OK;
}

mrcm_status mrcm_set_robin(mrcm_ctx* c, mrcm_beta_mode mode, double mbf, double smooth) {
  if (!c) return MRCM_EINVAL;
  if (mode != MRCM_BETA_ALPHA && mode != MRCM_BETA_CONST) return fail(c, MRCM_EINVAL, "bad beta mode");
  if (!(mbf > 0.0) || !(smooth > 0.0) || !std::isfinite(mbf) || !std::isfinite(smooth))
    return fail(c, MRCM_EINVAL, "Robin parameters must be positive and finite");
  const bool lu0 = auto_prefers_lu(c);
  c->beta_mode = mode;
  c->beta_mbf = mbf;
  c->beta_sm = smooth;
  // the automatic interface solver may change with the parameter
  invalidate(c, c->iface_solver == MRCM_IFACE_AUTO && lu0 != auto_prefers_lu(c));
  return MRCM_OK;
}

mrcm_status mrcm_set_precision(mrcm_ctx* c, mrcm_precision prec, double tol, int max_refine) {
  if (!c) return MRCM_EINVAL;
  if (prec != MRCM_FP64 && prec != MRCM_FP32_REFINE) return fail(c, MRCM_EINVAL, "bad precision");
  if (prec == MRCM_FP32_REFINE && (!(tol > 0.0) || max_refine < 0))
    return fail(c, MRCM_EINVAL, "refinement needs tol > 0 and max_refine >= 0");
  c->prec = prec;
  c->tol = tol;
  c->max_refine = max_refine;
  invalidate(c, false);
  return MRCM_OK;
}

mrcm_status mrcm_build_basis(mrcm_ctx* c) {
  if (!c) return MRCM_EINVAL;
  ++c->epoch;
  if (!c->have_k) return fail(c, MRCM_ESTATE, "permeability not set");
  if (!c->have_part) return fail(c, MRCM_ESTATE, "partition not set");
  if (!c->plan_valid) {
    mrcm_status st = make_plan(c);
    if (st) return st;
  }
  const bool r32 = c->prec == MRCM_FP32_REFINE;
  if (r32 && c->d3 &&
      (c->lds3f_basis > 150 * 1024 || c->lds3f_smooth > 150 * 1024 || c->lds3f_part > 150 * 1024))
    return fail(c, MRCM_EINVAL, "FP32 refinement: a 3-D box does not fit the LDS of a workgroup");
  if (r32 && !c->d3 && (!c->wave || c->lds32_basis > 150 * 1024 || c->lds32_smooth > 150 * 1024 ||
                        c->lds32_part > 150 * 1024))
    return fail(c, MRCM_EINVAL,
                "FP32 refinement is available for 2-D boxes with lines of <= 32 cells and 3-D boxes with "
                "planes of <= 64 cells");
  hipStream_t s = c->stream;
  if (c->timing) HIPCHK(c, hipEventRecord(c->ev[0], s));
  // a new solve clears the flags of the last one, unless they wait for
  // mrcm_wait (deferred errors)
  if (!c->flags_zero && !c->deferred) HIPCHK(c, hipMemsetAsync(c->flags, 0, sizeof(int), s));
  c->flags_zero = false;
  // K = exp(log K): inside the local kernels on the FP64 wave path and on
  // both 3-D paths
  if ((r32 && !c->d3) || !(c->wave || c->d3))
    HIPCHK(c, launch_exp(c->logk, c->K, c->kcomp * c->geo.ncells, c->flags, s));
  if (r32) {
    HIPCHK(c, hipMemsetAsync(c->d_iters, 0, sizeof(int), s));
    HIPCHK(c, hipMemsetAsync(c->d_resid, 0, sizeof(unsigned long long), s));
  }
  if (r32 && c->d3) {
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[8], s));
    HIPCHK(c, launch_basis3f(c->geo, c->d_obox, c->geo.nsub, c->d_seeds, c->logk, c->beta_mbf, c->fac32,
                             c->Pk, c->tr_u, c->tr_phi, c->tr_beta, 0, c->tol, c->max_refine, c->d_iters,
                             c->d_resid, c->flags, c->lds3f_basis, c->nw3_box, s));
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[9], s));
    HIPCHK(c, launch_particular3f(c->geo, c->d_pbox, c->geo.nsub, c->logk, c->K, c->f, c->bcv,
                                  c->beta_mbf, c->facp32, c->pbar, c->ubar, c->pibar, c->tol,
                                  c->max_refine, c->d_iters, c->d_resid, c->flags, c->lds3f_part,
                                  c->nw3_part, s));
  } else if (r32) {
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[8], s));
    HIPCHK(c, launch_local32_w(c->geo, c->d_obox, c->d_pbox, c->geo.nsub, c->d_seeds, c->K, c->f,
                               c->bcv, c->beta_mbf, c->fac32, c->facp32, c->Pk, c->tr_u, c->tr_phi,
                               c->tr_beta, c->pbar, c->ubar, c->pibar, c->tol, c->max_refine,
                               c->d_iters, c->d_resid, c->flags,
                               std::max(c->lds32_basis, c->lds32_part), s));
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[9], s));
  } else if (c->wave) {
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[8], s));
    HIPCHK(c, launch_local_w(c->geo, c->d_obox, c->d_pbox, c->geo.nsub, c->d_seeds, c->logk, c->K, c->f,
                             c->bcv, c->beta_mbf, c->fac, c->tco, c->facp, c->tcp, c->Pk, c->tr_u,
                             c->tr_phi, c->tr_beta, c->pbar, c->ubar, c->pibar, c->fact,
                             c->flags, std::max(c->lds_basis, 2 * c->lds_part + 16), c->lds_part, s));
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[9], s));
  } else if (c->d3) {
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[8], s));
    HIPCHK(c, launch_basis3(c->geo, c->d_obox, c->geo.nsub, c->d_seeds, c->logk, c->beta_mbf, c->fac,
                            c->Pk, c->tr_u, c->tr_phi, c->tr_beta, 0, c->flags, c->lds3_basis, c->nw3_box, s));
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[9], s));
    HIPCHK(c, launch_particular3(c->geo, c->d_pbox, c->geo.nsub, c->logk, c->K, c->f, c->bcv,
                                 c->beta_mbf, c->facp, c->pbar, c->ubar, c->pibar, c->flags,
                                 c->lds3_part, c->nw3_part, s));
  } else {
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[8], s));
    HIPCHK(c, launch_basis(c->geo, c->d_obox, c->geo.nsub, c->d_seeds, c->K, c->beta_mbf, c->fac,
                           c->scr, c->Pk, c->tr_u, c->tr_phi, c->tr_beta, c->flags, s));
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[9], s));
    HIPCHK(c, launch_particular(c->geo, c->d_pbox, c->geo.nsub, c->K, c->f, c->bcv, c->beta_mbf,
                                c->facp, c->scr, c->pbar, c->ubar, c->pibar, c->flags, s));
  }
  if (c->beta_sm != c->beta_mbf) {
    // Step 6: the smoothing Robin parameter differs, so the oversampled
    // boxes are factored once more with it
    auto grow = [&](auto*& ptr, long long count) -> hipError_t {
      if (ptr) return hipSuccess;
      return hipMalloc((void**)&ptr, std::max<long long>(count, 1) * sizeof(*ptr));
    };
    if (r32 && c->d3) {
      HIPCHK(c, grow(c->fac32s, c->fac_n));
      HIPCHK(c, launch_basis3f(c->geo, c->d_obox, c->geo.nsub, c->d_seeds, c->logk, c->beta_sm, c->fac32s,
                               c->Pk, c->tr_u, c->tr_phi, c->tr_beta, 1, c->tol, c->max_refine,
                               c->d_iters, c->d_resid, c->flags, c->lds3f_basis, c->nw3_box, s));
    } else if (r32) {
      HIPCHK(c, grow(c->fac32s, c->fac_n));
      HIPCHK(c, launch_factor32_w(c->geo, c->d_obox, c->geo.nsub, c->K, c->beta_sm, c->fac32s,
                                  c->d_iters, c->d_resid, c->flags, c->lds32_basis, s));
    } else if (c->wave) {
      HIPCHK(c, grow(c->facs, c->fac_n));
      HIPCHK(c, grow(c->facts, c->fac_n));
      HIPCHK(c, launch_factor_w(c->geo, c->d_obox, c->geo.nsub, c->logk, c->beta_sm, c->facs,
                                c->facts, c->flags, c->lds_factor, s));
    } else if (c->d3) {
      HIPCHK(c, grow(c->facs, c->fac_n));
      HIPCHK(c, launch_basis3(c->geo, c->d_obox, c->geo.nsub, c->d_seeds, c->logk, c->beta_sm,
                              c->facs, c->Pk, c->tr_u, c->tr_phi, c->tr_beta, 1, c->flags,
                              c->lds3_basis, c->nw3_box, s));
    } else {
      HIPCHK(c, grow(c->facs, c->fac_n));
      HIPCHK(c, launch_basis(c->geo, c->d_obox, c->geo.nsub, c->d_seeds, c->K, c->beta_sm, c->facs,
                             c->scr, c->Pk, c->tr_u, c->tr_phi, c->tr_beta, c->flags, s, 1));
    }
  }
  if (c->timing) HIPCHK(c, hipEventRecord(c->ev[1], s));
  c->timed_basis = c->timing;
  c->n_local_solves = c->nX + c->geo.nsub;
  c->state = 1;
  return MRCM_OK;
}

mrcm_status mrcm_solve_interface(mrcm_ctx* c) {
  if (!c) return MRCM_EINVAL;
  ++c->epoch;
  c->flags_zero = false;  // new flag-setting work may follow
  if (c->state < 1) return fail(c, MRCM_ESTATE, "basis not built");
  hipStream_t s = c->stream;
  if (c->timing) HIPCHK(c, hipEventRecord(c->ev[2], s));
  if (c->use_lsc && c->nX > 0) {
    // moments straight into the two-level solver's inner blocks and outer
    // coupling rows (set up first: zeros, identity padding, unit columns)
    HIPCHK(c, lsc_prepare(c->lsc, s));
    const BcrMap bm = lsc_map(c->lsc);
    HIPCHK(c, launch_moments(c->geo, c->d_ifc, (int)c->ifc.size(), c->mom_rows, c->d_basis,
                             c->d_seed_off, c->tr_u, c->tr_phi, c->tr_beta, c->ubar, c->pibar,
                             c->AB, c->ldab, c->kl, c->ku, c->rhs, s, &bm));
  } else if (c->use_bcr && c->nX > 0) {
    // moments straight into the reduction's layer blocks (set up first:
    // zero blocks and vectors, identity on the padding)
    HIPCHK(c, launch_bcr_init(c->bpool, c->bvec, c->d_lsize, c->bcr_M, c->bcr_bp, s));
    BcrMap bm;
    bm.row_lvl = c->d_row_lvl;
    bm.row_loc = c->d_row_loc;
    bm.col_lvl = c->d_col_lvl;
    bm.col_loc = c->d_col_loc;
    bm.M = c->bcr_M;
    bm.bp = c->bcr_bp;
    bm.pool = c->bpool;
    bm.vec = c->bvec;
    HIPCHK(c, launch_moments(c->geo, c->d_ifc, (int)c->ifc.size(), c->mom_rows, c->d_basis,
                             c->d_seed_off, c->tr_u, c->tr_phi, c->tr_beta, c->ubar, c->pibar,
                             c->AB, c->ldab, c->kl, c->ku, c->rhs, s, &bm));
  } else {
    HIPCHK(c, launch_fill(c->AB, 0.0, (long long)c->ldab * c->nX, s));
    HIPCHK(c, launch_moments(c->geo, c->d_ifc, (int)c->ifc.size(), c->mom_rows, c->d_basis,
                             c->d_seed_off, c->tr_u, c->tr_phi, c->tr_beta, c->ubar, c->pibar,
                             c->AB, c->ldab, c->kl, c->ku, c->rhs, s));
  }
  if (c->nX > 0) {
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[6], s));
    if (c->use_lsc) {
      HIPCHK(c, lsc_solve(c->lsc, c->X, c->flags, s));
    } else if (c->use_bcr) {
      mrcm_status st = bcr_solve(c, s);
      if (st) return st;
    } else {
      hipError_t e = launch_bandlu_solve(c->AB, c->ldab, c->nX, c->kl, c->ku, c->rhs, c->X,
                                         nullptr, c->flags, s);
      if (e == hipErrorInvalidValue)
        return fail(c, MRCM_EINVAL, "interface band (kl=%d, ku=%d) too wide for the LDS window",
                    c->kl, c->ku);
      HIPCHK(c, e);
    }
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[7], s));
  }
  HIPCHK(c, launch_combine(c->geo, c->d_seed_off, c->X, c->Pk, c->tr_u, c->pbar, c->ubar, c->p,
                           c->gflux, s));
  // the interface system's residual, row by row: the flux and pressure jump
  // moments of the MRCM-O state over the moments of the magnitudes of every
  // term of the row (a componentwise backward error); a row above the
  // tolerance (a breakdown of the solve, which does not pivot) raises
  // MRCM_ESINGULAR
  if (!c->ifc.empty()) {
    JumpTerms jt;
    jt.X = c->X;
    jt.seed_off = c->d_seed_off;
    jt.tr_u = c->tr_u;
    jt.tr_phi = c->tr_phi;
    jt.tr_beta = c->tr_beta;
    jt.ubar = c->ubar;
    jt.pibar = c->pibar;
    HIPCHK(c, launch_fill((double*)c->jmax_solve, 0.0, 2, s));
    HIPCHK(c, launch_jumps(c->geo, c->d_ifc, (int)c->ifc.size(), c->d_basis, c->K, c->p, c->gflux,
                           nullptr, c->jmax_solve, c->iface_check_tol, c->flags, s, &jt));
  }
  if (c->timing) HIPCHK(c, hipEventRecord(c->ev[3], s));
  c->timed_iface = c->timing;
  c->state = 2;
  c->n_ck = 0;
  c->n_phase = 0;
  return MRCM_OK;
}

}  // extern "C"

namespace {

// One smoothing sweep: the 2^d colour phases, in increasing colour order.
mrcm_status sweep(mrcm_ctx* c, hipStream_t s, int nt, double* p, double* gflux, bool ck = false) {
  const size_t np = (size_t)c->geo.ncells, ng = (size_t)c->geo.nsub * c->geo.gstride;
  for (int col = 0; col < (1 << c->d); ++col) {
    const int m0 = c->member_off[col], m1 = c->member_off[col + 1];
    if (ck) {
      // state before this phase, for the reverse pass
      HIPCHK(c, hipMemcpyAsync(c->ck_p + c->n_ck * np, p, np * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(c, hipMemcpyAsync(c->ck_g + c->n_ck * ng, gflux, ng * sizeof(double), hipMemcpyDeviceToDevice, s));
      ++c->n_ck;
    }
    const bool own = c->beta_sm != c->beta_mbf;  // Step 6 factors
    if (c->prec == MRCM_FP32_REFINE && c->d3) {
      HIPCHK(c, launch_smooth3f(c->geo, c->d_obox_col + m0, m1 - m0, c->K, c->f, c->bcv, c->beta_sm,
                                own ? c->fac32s : c->fac32, p, gflux, c->tol, c->max_refine, c->d_iters,
                                c->d_resid, c->flags, c->lds3f_smooth, c->nw3_box, c->smooth_cached, s));
    } else if (c->prec == MRCM_FP32_REFINE) {
      HIPCHK(c, launch_smooth32_w(c->geo, c->d_obox_col + m0, m1 - m0, c->K, c->f, c->bcv,
                                  c->beta_sm, own ? c->fac32s : c->fac32, p, gflux, c->tol,
                                  c->max_refine, c->d_iters, c->d_resid, c->flags,
                                  c->lds32_smooth, nt, s));
    } else if (c->wave) {
      HIPCHK(c, launch_smooth_w(c->geo, c->d_obox_col + m0, m1 - m0, c->K, c->f, c->bcv,
                                c->beta_sm, own ? c->facs : c->fac, own ? c->facts : c->fact,
                                c->tco, c->scr, p, gflux, c->lds_smooth, nt, s));
    } else if (c->d3) {
      HIPCHK(c, launch_smooth3(c->geo, c->d_obox_col + m0, m1 - m0, c->K, c->f, c->bcv, c->beta_sm,
                               own ? c->facs : c->fac, p, gflux, c->lds3_smooth, c->nw3_box, s));
    } else {
      HIPCHK(c, launch_smooth(c->geo, c->d_obox, c->d_members + m0, m1 - m0, c->K, c->f, c->bcv,
                              c->beta_sm, own ? c->facs : c->fac, nullptr, nullptr, c->scr, p,
                              gflux, c->prec, c->tol, c->max_refine, nullptr, nullptr, c->flags,
                              s));
    }
  }
  return MRCM_OK;
}

// Threads per box of the smoothing kernels: the requested value, or the
// fastest of 64, 128 and 256 over timed sweeps on copies of the current
// state; for 3-D boxes in the FP32 form, whether a box holds its plane
// inverses in registers (the variants give identical results).
mrcm_status tune_smoothing(mrcm_ctx* c, hipStream_t s) {
  if (c->smooth_nt) return MRCM_OK;
  const bool f3 = c->d3 && c->prec == MRCM_FP32_REFINE;
  if (!f3 && (c->smooth_nt_req || !c->wave)) {
    c->smooth_nt = c->smooth_nt_req ? c->smooth_nt_req : 256;
    return MRCM_OK;
  }
  const size_t np = (size_t)c->geo.ncells, ng = (size_t)c->geo.nsub * c->geo.gstride;
  if (!c->p_tune) HIPCHK(c, hipMalloc((void**)&c->p_tune, np * sizeof(double)));
  if (!c->gflux_tune) HIPCHK(c, hipMalloc((void**)&c->gflux_tune, std::max<size_t>(ng, 1) * sizeof(double)));
  HIPCHK(c, hipMemcpyAsync(c->p_tune, c->p, np * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->gflux_tune, c->gflux, ng * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipEventRecord(c->ev[10], s));
  float best = 0.f;
  int best_nt = 256, best_var = 8;
  const std::vector<int> cand = f3 ? std::vector<int>{8, 4, 2, 0} : std::vector<int>{64, 128, 256};
  for (int v : cand) {
    const int nt = f3 ? 256 : v;
    if (f3) c->smooth_cached = v;
    mrcm_status st = sweep(c, s, nt, c->p_tune, c->gflux_tune);  // warm-up
    if (st) return st;
    HIPCHK(c, hipEventRecord(c->ev[4], s));
    for (int r = 0; r < 3; ++r) {
      st = sweep(c, s, nt, c->p_tune, c->gflux_tune);
      if (st) return st;
    }
    HIPCHK(c, hipEventRecord(c->ev[5], s));
    HIPCHK(c, hipEventSynchronize(c->ev[5]));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[4], c->ev[5]));
    if (v == cand[0] || ms < best) {
      best = ms;
      best_nt = nt;
      best_var = v;
    }
  }
  if (f3) c->smooth_cached = best_var;
  HIPCHK(c, hipEventRecord(c->ev[11], s));
  HIPCHK(c, hipEventSynchronize(c->ev[11]));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev[10], c->ev[11]));
  c->ms_autotune = ms;
  c->smooth_nt = best_nt;
  return MRCM_OK;
}

// Capture nsteps sweeps into one graph (on a private stream), replayed by
// mrcm_smooth on the context's stream; kept until a call asks for another
// step count or the configuration changes.
mrcm_status capture_sweep(mrcm_ctx* c, int nsteps) {
  if (c->graph_exec && c->graph_steps == nsteps) return MRCM_OK;
  if (c->graph_exec) {
    HIPCHK(c, hipStreamSynchronize(c->stream));  // no replay of the old graph in flight
    drop_graph(c);
  }
  if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  mrcm_status st = MRCM_OK;
  for (int k = 0; k < nsteps && !st; ++k) st = sweep(c, c->cap_stream, c->smooth_nt, c->p, c->gflux);
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &gr);
  if (st) {
    if (gr) (void)hipGraphDestroy(gr);
    return st;
  }
  HIPCHK(c, e);
  c->graph = gr;
  HIPCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
  c->graph_steps = nsteps;
  return MRCM_OK;
}

}  // namespace

extern "C" {

mrcm_status mrcm_set_smoothing(mrcm_ctx* c, int use_graph, int threads_per_box) {
  if (!c) return MRCM_EINVAL;
  if (threads_per_box != 0 && threads_per_box != 64 && threads_per_box != 128 &&
      threads_per_box != 256)
    return fail(c, MRCM_EINVAL, "threads per box must be 0 (autotune), 64, 128 or 256");
  c->use_graph = use_graph != 0;
  c->smooth_nt_req = threads_per_box;
  c->smooth_nt = 0;
  drop_graph(c);
  return MRCM_OK;
}

mrcm_status mrcm_set_interface_check(mrcm_ctx* c, double tol) {
  if (!c) return MRCM_EINVAL;
  if (!(tol == tol)) return fail(c, MRCM_EINVAL, "tolerance is NaN");
  c->iface_check_tol = tol;
  return MRCM_OK;
}

mrcm_status mrcm_set_timing(mrcm_ctx* c, int on) {
  if (!c) return MRCM_EINVAL;
  c->timing = on != 0;
  return MRCM_OK;
}

mrcm_status mrcm_set_deferred_errors(mrcm_ctx* c, int on) {
  if (!c) return MRCM_EINVAL;
  if (c->deferred && !on) {
    c->deferred = false;
    return read_flags(c);  // what the deferred calls left
  }
  c->deferred = on != 0;
  return MRCM_OK;
}

mrcm_status mrcm_wait(mrcm_ctx* c) {
  if (!c) return MRCM_EINVAL;
  return read_flags(c);
}

mrcm_status mrcm_set_smoothing_persistent(mrcm_ctx* c, int on, int max_groups) {
  if (!c) return MRCM_EINVAL;
  if (max_groups < 0) return fail(c, MRCM_EINVAL, "max_groups < 0");
  c->persist = on != 0;
  c->persist_groups = max_groups;
  return MRCM_OK;
}

mrcm_status mrcm_smooth(mrcm_ctx* c, int nsteps) {
  if (!c) return MRCM_EINVAL;
  ++c->epoch;
  c->flags_zero = false;  // new flag-setting work may follow
  if (c->state < 2) return fail(c, MRCM_ESTATE, "interface not solved");
  if (nsteps < 0) return fail(c, MRCM_EINVAL, "nsteps < 0");
  hipStream_t s = c->stream;
  if (nsteps > 0) {
    mrcm_status st = tune_smoothing(c, s);
    if (st) return st;
    if (c->use_graph && !c->ckpt) {
      st = capture_sweep(c, nsteps);
      if (st) return st;
    }
  }
  if (c->ckpt && nsteps > 0) {
    // room for the checkpoints of these phases (grown with a copy)
    const int need = c->n_ck + (nsteps << c->d);
    if (need > c->ck_cap) {
      const size_t np = (size_t)c->geo.ncells, ng = (size_t)c->geo.nsub * c->geo.gstride;
      const int cap = std::max(need, 2 * c->ck_cap);
      double *np_ = nullptr, *ng_ = nullptr;
      HIPCHK(c, hipMalloc((void**)&np_, (size_t)cap * np * sizeof(double)));
      HIPCHK(c, hipMalloc((void**)&ng_, (size_t)cap * std::max<size_t>(ng, 1) * sizeof(double)));
      if (c->n_ck) {
        HIPCHK(c, hipMemcpyAsync(np_, c->ck_p, c->n_ck * np * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(ng_, c->ck_g, c->n_ck * ng * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));
      }
      dfree(c->ck_p);
      dfree(c->ck_g);
      c->ck_p = np_;
      c->ck_g = ng_;
      c->ck_cap = cap;
    }
  }
  const int nphase = nsteps << c->d;
  const bool try_grid = c->persist && c->wave && c->prec != MRCM_FP32_REFINE && !c->ckpt;
  if (c->timing) HIPCHK(c, hipEventRecord(c->ev[4], s));
  c->n_smooth_launches = nphase;
  c->n_smooth_phases = nphase;
  c->persist_used = false;
  if (try_grid && nphase > 0) {
    SmoothPhases ph;
    ph.ncol = 1 << c->d;
    for (int col = 0; col <= ph.ncol; ++col) ph.off[col] = c->member_off[col];
    const hipError_t e =
        launch_smooth_grid(c->geo, c->d_obox_col, ph, nphase, c->K, c->f, c->bcv, c->beta_sm,
                           c->beta_sm != c->beta_mbf ? c->facs : c->fac,
                           c->beta_sm != c->beta_mbf ? c->facts : c->fact, c->tco, c->p,
                           c->gflux, c->lds_smooth, c->smooth_nt, c->persist_groups, s);
    if (e == hipSuccess) {
      c->persist_used = true;
      c->n_smooth_launches = 1;
      nsteps = 0;  // all phases done
    } else if (e != hipErrorNotSupported && e != hipErrorCooperativeLaunchTooLarge) {
      HIPCHK(c, e);
    }
  }
  if (nsteps > 0 && c->use_graph && !c->ckpt) {
    HIPCHK(c, hipGraphLaunch(c->graph_exec, s));  // all nsteps sweeps
    nsteps = 0;
  }
  for (int step = 0; step < nsteps; ++step) {
    mrcm_status st = sweep(c, s, c->smooth_nt, c->p, c->gflux, c->ckpt);
    if (st) return st;
  }
  c->n_phase += nphase;
  if (c->timing) HIPCHK(c, hipEventRecord(c->ev[5], s));
  c->timed_smooth = c->timing;
  c->n_local_solves += (nphase >> c->d) * c->geo.nsub;
  return MRCM_OK;
}

mrcm_status mrcm_get_pressure(mrcm_ctx* c, double* p_dev) {
  if (!c) return MRCM_EINVAL;
  if (!p_dev) return fail(c, MRCM_EINVAL, "output is NULL");
  if (c->state < 2) return fail(c, MRCM_ESTATE, "no solution yet");
  HIPCHK(c, launch_pressure_out(c->geo, c->p, p_dev, c->partial, c->stream));
  return check_flags(c);
}

mrcm_status mrcm_get_flux(mrcm_ctx* c, double* flux_dev) {
  if (!c) return MRCM_EINVAL;
  if (!flux_dev) return fail(c, MRCM_EINVAL, "output is NULL");
  if (c->state < 2) return fail(c, MRCM_ESTATE, "no solution yet");
  HIPCHK(c, launch_flux_out(c->geo, c->K, c->p, c->gflux, c->bcv, flux_dev, c->stream));
  return check_flags(c);
}

mrcm_status mrcm_get_solution(mrcm_ctx* c, double* p_dev, double* flux_dev) {
  if (!c) return MRCM_EINVAL;
  if (!p_dev || !flux_dev) return fail(c, MRCM_EINVAL, "output is NULL");
  if (c->state < 2) return fail(c, MRCM_ESTATE, "no solution yet");
  HIPCHK(c, launch_solution_out(c->geo, c->K, c->p, c->gflux, c->bcv, p_dev, flux_dev, c->partial,
                                c->stream));
  return check_flags(c);
}

mrcm_status mrcm_get_coefficients(mrcm_ctx* c, double* x_dev) {
  if (!c) return MRCM_EINVAL;
  if (!x_dev) return fail(c, MRCM_EINVAL, "output is NULL");
  if (c->state < 2) return fail(c, MRCM_ESTATE, "no solution yet");
  if (c->nX > 0)
    HIPCHK(c, hipMemcpyAsync(x_dev, c->X, c->nX * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return check_flags(c);
}

mrcm_status mrcm_set_checkpointing(mrcm_ctx* c, int on) {
  if (!c) return MRCM_EINVAL;
  c->ckpt = on != 0;
  return MRCM_OK;
}

mrcm_status mrcm_adjoint(mrcm_ctx* c, const double* dJdp, const double* dJdflux, double* dJdlogK) {
  if (!c) return MRCM_EINVAL;
  ++c->epoch;
  c->flags_zero = false;  // new flag-setting work may follow
  if (!dJdlogK) return fail(c, MRCM_EINVAL, "output is NULL");
  if (c->state < 2) return fail(c, MRCM_ESTATE, "no solution to differentiate");
  if (!c->wave || c->d != 2)
    return fail(c, MRCM_EINVAL, "the adjoint needs 2-D boxes with lines of <= 32 cells");
  if (c->kcomp != 1) return fail(c, MRCM_EINVAL, "the adjoint needs a scalar permeability");
  if (!c->use_bcr)
    return fail(c, MRCM_EINVAL, "the adjoint needs the block-cyclic-reduction interface solver");
  if (c->n_ck != c->n_phase)
    return fail(c, MRCM_ESTATE, "smoothing ran without checkpointing (call mrcm_set_checkpointing first)");
  // the precision of the forward solve: FP64, or FP32 with FP64 refinement
  const bool r32 = c->prec == MRCM_FP32_REFINE;
  const size_t lds_sm = r32 ? c->lds_adj32_smooth : c->lds_adj_smooth;
  const size_t lds_bs = r32 ? c->lds_adj32_basis : c->lds_adj_basis;
  const size_t lds_pt = r32 ? c->lds_adj32_part : c->lds_adj_part;
  if (lds_bs > 150 * 1024 || lds_sm > 150 * 1024 || lds_pt > 150 * 1024)
    return fail(c, MRCM_EINVAL, "too many seeds per box for the adjoint kernels");
  if (c->beta_sm != c->beta_mbf)
    return fail(c, MRCM_EINVAL, "the adjoint needs equal Robin parameters in both stages");
  const Geo& g = c->geo;
  hipStream_t s = c->stream;
  const size_t N = (size_t)g.ncells, ng = std::max<size_t>((size_t)g.nsub * g.gstride, 1);
  const size_t nX = std::max(c->nX, 1), ntr = (size_t)nX * g.gstride;
  auto need = [&](double*& p, size_t n) -> mrcm_status {
    if (!p) HIPCHK(c, hipMalloc((void**)&p, n * sizeof(double)));
    return MRCM_OK;
  };
#define NEED(p, n) do { mrcm_status s_ = need(p, n); if (s_) return s_; } while (0)
  NEED(c->a_pb, N); NEED(c->a_gfb, ng); NEED(c->a_Kb, N); NEED(c->a_Xb, nX); NEED(c->a_nu, nX);
  NEED(c->a_trub, ntr); NEED(c->a_trphib, ntr); NEED(c->a_trbetab, ng); NEED(c->a_ubarb, ng);
  NEED(c->a_pibarb, ng); NEED(c->a_mean, 1);
#undef NEED
  if (!c->d_seed_sub) {
    std::vector<int> ss(nX, 0);
    for (int i = 0; i < g.nsub; ++i)
      for (int k = c->seed_off[i]; k < c->seed_off[i + 1]; ++k) ss[k] = i;
    HIPCHK(c, hipMalloc((void**)&c->d_seed_sub, nX * sizeof(int)));
    HIPCHK(c, hipMemcpy(c->d_seed_sub, ss.data(), nX * sizeof(int), hipMemcpyHostToDevice));
  }
  // the flags are not cleared here: they may still hold an error of the
  // forward solve that no call has read yet (deferred errors, or no output
  // call since it), which this call or mrcm_wait must report
  // outputs
  HIPCHK(c, launch_fill(c->a_gfb, 0.0, (long long)ng, s));
  HIPCHK(c, launch_adj_out(g, c->K, c->p, c->bcv, dJdp, dJdflux, c->a_mean, c->a_pb, c->a_gfb,
                           c->a_Kb, s));
  // FP32 form: cached FP32 factors of the seed / smoothing boxes (equal
  // Robin parameters: one set) and of the particular boxes
  const Adj32 a32 = {c->fac32, c->tol, c->max_refine, c->d_iters, c->d_resid, c->flags};
  const Adj32 a32p = {c->facp32, c->tol, c->max_refine, c->d_iters, c->d_resid, c->flags};
  // smoothing phases, last first
  const size_t np = N;
  for (int ph = c->n_ck - 1; ph >= 0; --ph) {
    const int col = ph % (1 << g.d);
    const int m0 = c->member_off[col], m1 = c->member_off[col + 1];
    HIPCHK(c, launch_adj_smooth(g, c->d_obox, c->d_members + m0, m1 - m0, c->K, c->f, c->bcv,
                                c->beta_sm, c->fac, c->fact, c->tco, r32 ? &a32 : nullptr,
                                c->ck_p + ph * np, c->ck_g + ph * ng, c->a_pb, c->a_gfb, c->a_Kb,
                                lds_sm, s));
  }
  // MRCM-O assembly
  HIPCHK(c, launch_adj_combine(g, c->d_seed_sub, c->nX, c->X, c->Pk, c->tr_u, c->a_pb, c->a_gfb,
                               c->a_Xb, c->a_trub, s));
  // interface system, transposed: G^T nu = Xbar by the same reduction
  {
    const int M = c->bcr_M, bp = c->bcr_bp;
    const long long bs = (long long)bp * bp;
    HIPCHK(c, launch_fill(c->AB, 0.0, (long long)(c->kl + c->ku + 1) * c->nX, s));
    HIPCHK(c, launch_moments(g, c->d_ifc, (int)c->ifc.size(), c->mom_rows, c->d_basis, c->d_seed_off, c->tr_u,
                             c->tr_phi, c->tr_beta, c->ubar, c->pibar, c->AB, c->ldab, c->kl, c->ku,
                             c->rhs, s));
    (void)bs;
    HIPCHK(c, launch_bcr_init(c->bpool, c->bvec, c->d_lsize, M, bp, s));
    HIPCHK(c, launch_bcr_scatter_t(c->AB, c->a_Xb, c->nX, c->kl, c->ku, c->d_row_lvl, c->d_row_loc,
                                   c->d_col_lvl, c->d_col_loc, M, bp, c->bpool, c->bvec, s));
    {
      mrcm_status st = run_bcr_ops(c, s);
      if (st) return st;
    }
    HIPCHK(c, launch_bcr_gather_t(c->bvec + 2LL * M * bp, c->d_row_lvl, c->d_row_loc, c->nX, bp,
                                  c->a_nu, s));
  }
  // moments
  HIPCHK(c, hipMemcpyAsync(c->a_ubarb, c->a_gfb, ng * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, launch_fill(c->a_trphib, 0.0, (long long)ntr, s));
  HIPCHK(c, launch_fill(c->a_trbetab, 0.0, (long long)ng, s));
  HIPCHK(c, launch_fill(c->a_pibarb, 0.0, (long long)ng, s));
  HIPCHK(c, launch_adj_moments(g, c->d_ifc, (int)c->ifc.size(), c->d_basis, c->d_seed_off, c->X,
                               c->a_nu, c->tr_u, c->tr_beta, c->a_trub, c->a_trphib, c->a_trbetab,
                               c->a_ubarb, c->a_pibarb, s));
  // seeds and particular problems
  HIPCHK(c, launch_adj_basis(g, c->d_obox, g.nsub, c->d_seeds, c->K, c->beta_mbf, c->fac, c->fact,
                             r32 ? &a32 : nullptr, c->X, c->a_pb, c->tr_u, c->a_trub, c->a_trphib,
                             c->a_trbetab, c->a_Kb, lds_bs, s));
  HIPCHK(c, launch_adj_particular(g, c->d_pbox, g.nsub, c->K, c->bcv, c->beta_mbf, c->facp,
                                  r32 ? &a32p : nullptr, c->pbar, c->a_pb, c->a_ubarb, c->a_pibarb,
                                  c->a_Kb, lds_pt, s));
  HIPCHK(c, launch_adj_logk(c->K, c->a_Kb, g.ncells, dJdlogK, s));
  return check_flags(c);
}

mrcm_status mrcm_get_balance(mrcm_ctx* c, double* cell_residual_dev, double* jumps_dev,
                             mrcm_balance* out) {
  if (!c) return MRCM_EINVAL;
  if (!out) return fail(c, MRCM_EINVAL, "output is NULL");
  if (c->state < 2) return fail(c, MRCM_ESTATE, "no solution yet");
  const Geo& g = c->geo;
  hipStream_t s = c->stream;
  HIPCHK(c, launch_cell_balance(g, c->K, c->p, c->gflux, c->bcv, c->f, cell_residual_dev,
                                c->bal_partial, std::max(cell_balance_blocks(g), 256), c->bal_out, s));
  HIPCHK(c, launch_fill((double*)c->jmax_bal, 0.0, 2, s));
  HIPCHK(c, launch_jumps(g, c->d_ifc, (int)c->ifc.size(), c->d_basis, c->K, c->p, c->gflux,
                         jumps_dev, c->jmax_bal, 0.0, c->flags, s));
  double v[kBalParts];
  unsigned long long jm[2];
  HIPCHK(c, hipMemcpyAsync(v, c->bal_out, sizeof v, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(jm, c->jmax_bal, sizeof jm, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  std::memset(out, 0, sizeof *out);
  out->mass_residual_max = v[0];
  out->mass_residual_rel = v[1] > 0.0 ? v[0] / v[1] : v[0];
  out->source_total = v[2];
  double tot = 0.0;
  for (int q = 0; q < 6; ++q) {
    out->outflow[q] = q < 2 * g.d ? v[3 + q] : 0.0;
    tot += out->outflow[q];
  }
  out->outflow_total = tot;
  std::memcpy(&out->flux_jump_max, &jm[0], sizeof(double));
  std::memcpy(&out->pressure_jump_max, &jm[1], sizeof(double));
  return check_flags(c);
}

mrcm_status mrcm_get_balance_static(mrcm_ctx* c, double* cell_residual_dev, double* jumps_dev,
                                    mrcm_balance* out) {
  if (!c) return MRCM_EINVAL;
  if (!out) return fail(c, MRCM_EINVAL, "output is NULL");
  // scratch layout: jump maxima (2), results (16), partial sums of the
  // 256-cell workgroups
  const long long ncells = (long long)c->n[0] * c->n[1] * c->n[2];
  const long long need = 18 + (ncells + 255) / 256 * kBalParts;
  if (need > kStaticScratchDoubles)
    return fail(c, MRCM_EINVAL,
                "grid of %lld cells needs %lld doubles of static scratch, more than the %d available "
                "(at most %d cells)", ncells, need, kStaticScratchDoubles,
                (kStaticScratchDoubles - 18) / kBalParts * 256);
  if (c->state < 2) return fail(c, MRCM_ESTATE, "no solution yet");
  const Geo& g = c->geo;
  double* sc = nullptr;
  HIPCHK(c, static_scratch(&sc));
  hipStream_t s = c->stream;
  unsigned long long* jm = reinterpret_cast<unsigned long long*>(sc);
  double* res = sc + 2;
  double* part = sc + 18;
  HIPCHK(c, launch_cell_balance(g, c->K, c->p, c->gflux, c->bcv, c->f, cell_residual_dev, part,
                                cell_balance_blocks(g), res, s));
  HIPCHK(c, launch_fill(sc, 0.0, 2, s));  // the maxima start at zero
  HIPCHK(c, launch_jumps(g, c->d_ifc, (int)c->ifc.size(), c->d_basis, c->K, c->p, c->gflux,
                         jumps_dev, jm, 0.0, c->flags, s));
  HIPCHK(c, hipMemcpyAsync(c->stage_host, sc, (2 + kBalParts) * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const double* v = c->stage_host + 2;
  std::memset(out, 0, sizeof *out);
  out->mass_residual_max = v[0];
  out->mass_residual_rel = v[1] > 0.0 ? v[0] / v[1] : v[0];
  out->source_total = v[2];
  double tot = 0.0;
  for (int q = 0; q < 6; ++q) {
    out->outflow[q] = q < 2 * g.d ? v[3 + q] : 0.0;
    tot += out->outflow[q];
  }
  out->outflow_total = tot;
  std::memcpy(&out->flux_jump_max, c->stage_host, sizeof(double));
  std::memcpy(&out->pressure_jump_max, c->stage_host + 1, sizeof(double));
  return check_flags(c);
}

mrcm_status mrcm_rel_error(mrcm_ctx* c, const double* p_ref_dev, const double* flux_ref_dev,
                           double* out) {
  if (!c) return MRCM_EINVAL;
  if (!out) return fail(c, MRCM_EINVAL, "output is NULL");
  if (c->state < 2) return fail(c, MRCM_ESTATE, "no solution yet");
  const Geo& g = c->geo;
  hipStream_t s = c->stream;
  const long long N = g.ncells, NF = N * 2 * g.d;
  if (!c->cmp_p) HIPCHK(c, hipMalloc((void**)&c->cmp_p, N * sizeof(double)));
  if (!c->cmp_f) HIPCHK(c, hipMalloc((void**)&c->cmp_f, NF * sizeof(double)));
  HIPCHK(c, launch_solution_out(g, c->K, c->p, c->gflux, c->bcv, c->cmp_p, c->cmp_f, c->partial, s));
  out[0] = out[1] = NAN;
  double r[4] = {0, 0, 0, 0};
  if (p_ref_dev) HIPCHK(c, launch_sq_dist(c->cmp_p, p_ref_dev, N, c->bal_partial, c->bal_out, s));
  if (p_ref_dev) HIPCHK(c, hipMemcpyAsync(r, c->bal_out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (flux_ref_dev) {
    HIPCHK(c, launch_sq_dist(c->cmp_f, flux_ref_dev, NF, c->bal_partial, c->bal_out, s));
    HIPCHK(c, hipMemcpyAsync(r + 2, c->bal_out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
  }
  if (p_ref_dev) out[0] = std::sqrt(r[0]) / std::sqrt(r[1]);
  if (flux_ref_dev) out[1] = std::sqrt(r[2]) / std::sqrt(r[3]);
  return check_flags(c);
}

mrcm_status mrcm_get_stats(mrcm_ctx* c, mrcm_stats* out) {
  if (!c) return MRCM_EINVAL;
  if (!out) return fail(c, MRCM_EINVAL, "output is NULL");
  std::memset(out, 0, sizeof *out);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  out->n_subdomains = c->geo.nsub;
  out->n_boxes = c->geo.nsub;
  out->n_unknowns = c->nX;
  out->band_kl = c->kl;
  out->band_ku = c->ku;
  out->interface_solver = c->use_lsc ? MRCM_IFACE_LAYERED : (c->use_bcr ? MRCM_IFACE_BCR : MRCM_IFACE_BAND_LU);
  out->n_local_solves = c->n_local_solves;
  out->bytes_factor = (double)(c->fac_n + c->facp_n) *
                      (c->prec == MRCM_FP32_REFINE ? sizeof(float) : sizeof(double));
  if (c->wave && c->prec != MRCM_FP32_REFINE) {
    // one symmetric inverse per block, stored as its lower triangle
    double n = 0.0;
    for (const Box& B : c->obox) n += (double)B.nblk * B.nb * (B.nb + 1) / 2;
    for (const Box& B : c->pbox) n += (double)B.nblk * B.nb * (B.nb + 1) / 2;
    out->bytes_factor = n * sizeof(double);
  }
  if (c->plan_valid && c->prec == MRCM_FP32_REFINE) {
    int it = 0;
    unsigned long long rb = 0;
    HIPCHK(c, hipMemcpy(&it, c->d_iters, sizeof it, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&rb, c->d_resid, sizeof rb, hipMemcpyDeviceToHost));
    out->refine_max_iters = it;
    double r;
    std::memcpy(&r, &rb, sizeof r);
    out->refine_max_resid = r;
  }
  float ms = 0.f;
  if (c->timed_basis && hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) out->ms_basis = ms;
  if (c->timed_iface && hipEventElapsedTime(&ms, c->ev[2], c->ev[3]) == hipSuccess) out->ms_interface = ms;
  if (c->timed_smooth && hipEventElapsedTime(&ms, c->ev[4], c->ev[5]) == hipSuccess) out->ms_smooth = ms;
  if (c->timed_iface && c->nX > 0 && hipEventElapsedTime(&ms, c->ev[6], c->ev[7]) == hipSuccess)
    out->ms_interface_solve = ms;
  if (c->timed_basis && hipEventElapsedTime(&ms, c->ev[8], c->ev[9]) == hipSuccess)
    out->ms_basis_kernel = ms;
  out->n_smooth_launches = c->n_smooth_launches;
  out->smooth_threads = c->smooth_nt;
  out->smooth_cached = c->d3 && c->prec == MRCM_FP32_REFINE ? c->smooth_cached : 0;
  out->smooth_graph = c->use_graph ? 1 : 0;
  out->ms_autotune = c->ms_autotune;
  out->n_smooth_phases = c->n_smooth_phases;
  out->smooth_persistent = c->persist_used ? 1 : 0;
  out->interface_residual = 0.0;
  if (c->plan_valid && c->state >= 2 && !c->ifc.empty()) {
    unsigned long long jm[2];
    HIPCHK(c, hipMemcpy(jm, c->jmax_solve, sizeof jm, hipMemcpyDeviceToHost));
    double a, b;
    std::memcpy(&a, &jm[0], sizeof a);
    std::memcpy(&b, &jm[1], sizeof b);
    out->interface_residual = std::max(a, b);
  }
  return check_flags(c);
}

const char* mrcm_last_error(const mrcm_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

mrcm_status mrcm_destroy(mrcm_ctx* c) {
  if (!c) return MRCM_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  free_plan(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  dfree(c->logk); dfree(c->K); dfree(c->f); dfree(c->bcv); dfree(c->flags);
  if (c->flags_host) (void)hipHostFree(c->flags_host);
  if (c->stage_host) (void)hipHostFree(c->stage_host);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return MRCM_OK;
}

}  // extern "C"
