/*
 * mrcm.h -- C ABI of the MI355X (gfx950) MRCM-OS hot path.
 *
 * The library solves single-phase Darcy flow (u = -K grad p, div u = f,
 * p = g or u.n = z on the boundary; paper Section 2, equations eq1a-eq1d) on
 * a uniform Cartesian grid with the oversampled Multiscale Robin Coupled
 * Method with smoothing of Zhou, Guiraldello and Pereira (arXiv 2404.13811):
 *
 *   mrcm_build_basis      Algorithm 1, Steps 1-2 (+ the particular problems of
 *                         Step 4): batched local factorisations on the
 *                         oversampled boxes and on the subdomains, the seed
 *                         solves that define the informed spaces (equation
 *                         informed_space) and the multiscale basis functions.
 *   mrcm_solve_interface  Steps 3-5: interface system (equations int_ujump,
 *                         int_pjump) assembled on the device, solved in FP64
 *                         on the device, MRCM-O solution assembled.
 *   mrcm_smooth           Steps 6-7 / Section 3: colored Robin re-solves on
 *                         the oversampled boxes with cached factors.
 *   mrcm_get_pressure / mrcm_get_flux   outputs.
 *
 * Conventions
 *   - Cells are numbered x fastest; axis 0 = x.  A grid has ncell[0..dim-1]
 *     cells of size h (cubic).  Domain sides are 0..2*dim-1 =
 *     (-x, +x, -y, +y, -z, +z); boundary values of side s are given per face
 *     in the x-fastest order of the cells that touch that side.
 *   - Every array argument is a DEVICE pointer (hipMalloc'd or a torch CUDA
 *     tensor's data_ptr) owned by the caller, FP64, contiguous.  Inputs are
 *     copied into library workspace during the call, so the caller may free
 *     or reuse them afterwards.  Outputs are written by work enqueued on the
 *     context's stream; synchronise that stream before reading them.
 *   - The library owns all workspace (factors, basis functions, interface
 *     system); it is released by mrcm_destroy.
 *   - Every function returns an mrcm_status and never aborts; on failure
 *     mrcm_last_error() holds a human-readable message.
 *   - Call order: create -> set_* -> build_basis -> solve_interface ->
 *     smooth* -> get_*.  A set_* call after build_basis invalidates the
 *     basis; a call made too early returns MRCM_ESTATE.
 *   - One context per stream; contexts share no state.  Calls on one context
 *     must not overlap in time (not thread-safe per context).
 */
#ifndef MRCM_H
#define MRCM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrcm_ctx mrcm_ctx;

typedef enum {
  MRCM_OK = 0,
  MRCM_EINVAL = 1,     /* bad argument (null pointer, bad size, K <= 0, ...)  */
  MRCM_ENOMEM = 2,     /* device allocation failed                            */
  MRCM_EDEVICE = 3,    /* a HIP call or kernel launch failed                  */
  MRCM_ESTATE = 4,     /* call out of order                                   */
  MRCM_ENOTPD = 5,     /* a local factorisation met a non-positive pivot      */
  MRCM_ENOCONV = 6,    /* iterative refinement did not reach its tolerance    */
  MRCM_EINCOMPAT = 7,  /* pure-Neumann problem with non-zero net source       */
  MRCM_ESINGULAR = 8   /* interface system singular (zero pivot)              */
} mrcm_status;

/* Interface spaces M_H = V_H and seed family of Lambda_H^i (paper Section 2:
 * piecewise constant or piecewise linear per coarse interface).  FINE uses
 * one indicator per fine face (the setting of Proposition 2); it exists to
 * test the path against the fine-grid solution. */
typedef enum { MRCM_SPACE_CONST = 0, MRCM_SPACE_LINEAR = 1, MRCM_SPACE_FINE = 2 } mrcm_space;

/* Robin parameter: ALPHA -> beta = alpha * H / K_H per face (paper, equation
 * after genRobin; H = subdomain width along the face normal, K_H = harmonic
 * mean of the two adjacent cells); CONST -> beta = the given value. */
typedef enum { MRCM_BETA_ALPHA = 0, MRCM_BETA_CONST = 1 } mrcm_beta_mode;

/* FP64: local factors and solves in FP64.  FP32_REFINE: local factors and
 * solves in FP32 on the diagonally scaled local matrices, corrected by FP64
 * iterative refinement with the residual r = b - A x evaluated from K in
 * FP64 until the componentwise backward error max_c |r_c| / (|A||x| + |b|)_c
 * is <= tol (at most max_refine corrections; MRCM_ENOCONV otherwise).
 * Available for 2-D boxes whose lines have at most 32 cells and for 3-D
 * boxes whose planes have at most 64 cells (otherwise mrcm_build_basis
 * returns MRCM_EINVAL). */
typedef enum { MRCM_FP64 = 0, MRCM_FP32_REFINE = 1 } mrcm_precision;

typedef enum { MRCM_BC_NEUMANN = 0, MRCM_BC_DIRICHLET = 1 } mrcm_bc_type;

/* Direct solver of the interface system (Algorithm 1, Step 5), both FP64 on
 * the device.  BAND_LU: banded LU with partial pivoting in the natural
 * (interface-major) equation order, one workgroup.  BCR: block cyclic
 * reduction over the layers of subdomains along the last axis, with the
 * flux equations of an interface assigned to its lower-indexed subdomain and
 * the pressure equations to the higher one (square layer blocks, block
 * tridiagonal system), dense block inverses without pivoting; needs layer
 * blocks of at most 256 unknowns.  AUTO: BCR when it applies, else LAYERED
 * on 3-D grids, else BAND_LU;
 * BAND_LU also when the basis Robin parameter is alpha > 1e4 (MRCM_BETA_ALPHA),
 * where the reduction without pivoting loses accuracy (measured: backward
 * error 1e-9 at alpha = 1e4, breakdown from 1e6 on). */
typedef enum {
  MRCM_IFACE_AUTO = 0,
  MRCM_IFACE_BAND_LU = 1,
  MRCM_IFACE_BCR = 2,
  /* 3-D grids: two-level reduction.  Outer layers of subdomains along the
   * axis with the most subdomains; the block tridiagonal system of every
   * outer layer (over inner layers of one row of subdomains, blocks of at
   * most 256 unknowns) is reduced for all layers at once with its couplings
   * to the neighbouring layers as extra right-hand sides; the reduced system
   * over the gaps between outer layers (one dense block per gap) is solved by
   * block cyclic reduction with recursive two-by-two block inverses.  Exact
   * elimination, no pivoting. */
  MRCM_IFACE_LAYERED = 3
} mrcm_iface_solver;

typedef struct {
  int n_subdomains;        /* m                                              */
  int n_boxes;             /* oversampled boxes (= m)                        */
  int n_unknowns;          /* interface unknowns sum_i dim Lambda_H^i        */
  int band_kl, band_ku;    /* bandwidths of the interface system             */
  int n_local_solves;      /* right-hand sides solved so far                 */
  int refine_max_iters;    /* most FP32 solves used by one refined system     */
  double refine_max_resid; /* largest final componentwise backward error      */
  double ms_basis, ms_interface, ms_smooth;  /* device time of the last calls */
  double bytes_factor;     /* bytes of cached local factors                  */
  double ms_interface_solve; /* device time of the interface factor + solve  */
  int interface_solver;    /* MRCM_IFACE_BAND_LU, _BCR or _LAYERED in use      */
  int n_smooth_launches;   /* colour-phase launches of the last mrcm_smooth    */
  double ms_basis_kernel;  /* device time of the seed-solve kernel alone       */
  int smooth_threads;      /* threads per box of the smoothing kernels         */
  int smooth_graph;        /* 1: sweeps replay a captured graph                */
  double ms_autotune;      /* device time of the last smoothing autotune       */
  int n_smooth_phases;     /* colour phases run by the last mrcm_smooth        */
  int smooth_persistent;   /* 1: the last mrcm_smooth ran as one cooperative
                              launch                                          */
  double interface_residual; /* residual check of the last interface solve:
                              the componentwise backward error
                              max_r |G X - r|_r / (|G| |X| + |r|)_r of the
                              interface system (Algorithm 1, Step 5), from the
                              flux and pressure jump moments of the MRCM-O
                              state; above the check tolerance (default 1e-5,
                              mrcm_set_interface_check) the solve raises
                              MRCM_ESINGULAR.  0 if no interface.            */
  int smooth_cached;       /* 3-D boxes in the FP32 form: the planes (8, 4, 2
                              or 0) whose inverses a smoothing box holds in
                              registers across its refinement sweeps; the
                              others are read from memory by every sweep
                              (the fastest variant, timed by the autotuner)   */
} mrcm_stats;

/* Conservation and continuity measures of the current solution (Section 5's
 * error measures; the cell mass balance of the mixed system, eq1b, and the
 * interface equations int_ujump and int_pjump).  u is the output velocity
 * of mrcm_get_flux; on an interface Gamma_ij each subdomain's own outward
 * flux u_i, u_j and pressure trace pi = p_c - u h / (2 K_c) are used. */
typedef struct {
  double mass_residual_max;  /* max over cells |sum_faces |e| u - f h^d|      */
  double mass_residual_rel;  /* the same over max over cells sum |e| |u|       */
  double source_total;       /* sum over cells of f h^d                        */
  double outflow[6];         /* per domain side: sum over its faces |e| u.n    */
  double outflow_total;      /* sum of outflow[]: source_total when conserved  */
  double flux_jump_max;      /* max over interfaces and test functions mu of
                                |sum |e| mu (u_i + u_j)| / sum |e||mu|(|u_i|+|u_j|) */
  double pressure_jump_max;  /* the same for pi_i - pi_j                        */
} mrcm_balance;

/* Create a context for a dim-dimensional grid (dim = 2 or 3) of
 * ncell[0..dim-1] cells of size h.  stream: a hipStream_t (NULL = default
 * stream) on which all work of this context is enqueued.
 * Errors: MRCM_EINVAL (dim, ncell or h out of range, out == NULL),
 * MRCM_EDEVICE. */
mrcm_status mrcm_create(int dim, const int* ncell, double h, void* stream, mrcm_ctx** out);

/* A batch of nbatch independent 2-D problems that share the grid
 * (ncell[0] x ncell[1] cells of size h) and every setting of the context
 * (partition, spaces, Robin parameters, precision, solver) but not the data:
 * each member has its own log K, source and boundary values.  Every stage
 * runs the whole batch at once: one launch of the local kernels over all
 * members' boxes, one launch per colour phase of the smoothing sweep, one
 * interface solve (the members' systems are independent blocks of it, the
 * MRCM-OS of Algorithm 1 applied to each member; every step but Step 5 is
 * per subdomain, Section 4), one adjoint.
 * Layout: member-major everywhere.  Per-cell arrays (log K, f, pressure,
 * gradients) hold nbatch * ncell[0] * ncell[1] values, member m's cells at
 * m * ncell[0] * ncell[1] (x fastest within a member); per-face fluxes
 * 4 values per cell in the same order; the boundary values of the x sides
 * (sides 0, 1) nbatch * ncell[1] values and of the y sides (2, 3)
 * nbatch * ncell[0], member after member.  Equivalently the members are
 * stacked along y into one grid of ncell[0] x nbatch * ncell[1] cells that
 * is cut between members: no cell, box or interface couples two members.
 * Interface unknowns (mrcm_get_coefficients) follow the members in order.
 * Requires dim = 2, nbatch >= 1, a pressure (Dirichlet) boundary on some
 * side (mrcm_build_basis: MRCM_EINVAL otherwise, the members would need
 * their own gauge) and ncell[1] a multiple of the subdomain size along y
 * (mrcm_set_partition: MRCM_EINVAL).  mrcm_get_balance and mrcm_rel_error
 * report over the whole batch.  Errors as mrcm_create, and MRCM_EINVAL for
 * dim != 2 with nbatch > 1 or nbatch < 1. */
mrcm_status mrcm_create_batched(int dim, const int* ncell, double h, int nbatch, void* stream,
                                mrcm_ctx** out);

/* log K per cell (N values, x fastest; paper eq1a, scalar K).  Copied.
 * Errors: MRCM_EINVAL on NULL; non-finite values are detected at
 * mrcm_build_basis (MRCM_EINVAL). */
mrcm_status mrcm_set_permeability(mrcm_ctx* ctx, const double* logk_dev);

/* Diagonal permeability tensor K = diag(K_x, K_y[, K_z]) per cell (paper
 * Section 2: eq1a with K symmetric positive definite): log K as dim x N
 * values, component-major (the dim components of axis 0, then axis 1, ...;
 * each x fastest; for a batch, each component over all members in order).
 * On the two-point flux a face normal to axis a sees only K_a: in its
 * transmissibility, its Robin and Dirichlet coefficients, beta = alpha H /
 * (K_a)_H and the half-cell pressure trace.  Copied; replaces a scalar K
 * and is replaced by mrcm_set_permeability.  Every forward path takes it;
 * mrcm_adjoint refuses it (MRCM_EINVAL: the gradient is with respect to a
 * scalar log K).  The box layouts hold one permeability tile per
 * component, so 3-D boxes need 2 more halo tiles of LDS.  Errors as
 * mrcm_set_permeability. */
mrcm_status mrcm_set_permeability_diag(mrcm_ctx* ctx, const double* logk_dev);

/* Source density f per cell (eq1b; N values) or NULL for f = 0.  Copied. */
mrcm_status mrcm_set_source(mrcm_ctx* ctx, const double* f_dev);

/* Boundary condition of domain side `side` (0..2*dim-1): pressure g (eq. for
 * p on the pressure boundary) or outward normal velocity z (eq1d), one value
 * per boundary face, or val_dev == NULL for zero.  Default: Neumann, z = 0. */
mrcm_status mrcm_set_bc(mrcm_ctx* ctx, int side, mrcm_bc_type type, const double* val_dev);

/* Non-overlapping partition into boxes of sub[a] cells per axis (ncell[a]
 * must be a multiple of sub[a]) and oversampling width `overlap` cells,
 * 0 <= overlap <= min(sub) - 1 (paper Section 2, Figure of the two
 * partitions; oversampled boxes are clipped to the domain). */
mrcm_status mrcm_set_partition(mrcm_ctx* ctx, const int* sub, int overlap);

mrcm_status mrcm_set_interface_space(mrcm_ctx* ctx, mrcm_space space);

/* Interface solver (default MRCM_IFACE_AUTO).  Errors: MRCM_EINVAL; with
 * MRCM_IFACE_BCR, mrcm_build_basis fails with MRCM_EINVAL when the layer
 * blocks are not square or exceed 256 unknowns. */
mrcm_status mrcm_set_interface_solver(mrcm_ctx* ctx, mrcm_iface_solver solver);

/* Robin parameters of the basis functions (Algorithm 1, Steps 1-2, and the
 * particular problems of Step 4) and of the smoothing steps (Steps 6-7;
 * Section 3 allows any positive value).  Values > 0.  When they differ,
 * mrcm_build_basis also runs Step 6: every oversampled box is factored a
 * second time with the smoothing parameter, and mrcm_smooth uses those
 * factors (one more set of cached factors in device memory).  The adjoint
 * needs equal values. */
mrcm_status mrcm_set_robin(mrcm_ctx* ctx, mrcm_beta_mode mode, double mbf, double smooth);

/* Precision of the local factorisations and solves.  tol > 0 and
 * max_refine >= 0 are used by MRCM_FP32_REFINE only. */
mrcm_status mrcm_set_precision(mrcm_ctx* ctx, mrcm_precision prec, double tol, int max_refine);

/* Algorithm 1, Steps 1-2 and the particular problems of Step 4.
 * Errors: MRCM_ESTATE (inputs missing), MRCM_EINVAL (bad K),
 * MRCM_EINCOMPAT, MRCM_ENOTPD, MRCM_ENOCONV, MRCM_ENOMEM, MRCM_EDEVICE. */
mrcm_status mrcm_build_basis(mrcm_ctx* ctx);

/* Steps 3-5: interface system and MRCM-O solution (resets smoothing).  The
 * solve is checked on the device: the componentwise backward error of every
 * interface equation (see mrcm_stats.interface_residual) must not exceed
 * the check tolerance (default 1e-5), else the solve's device error is
 * MRCM_ESINGULAR (reported by the next call that reads the device flags).
 * Errors: MRCM_ESTATE, MRCM_ESINGULAR, MRCM_EDEVICE. */
mrcm_status mrcm_solve_interface(mrcm_ctx* ctx);

/* Steps 6-7: nsteps >= 0 further smoothing steps on the current solution
 * (re-entrant: smooth(a); smooth(b) equals smooth(a + b)). */
mrcm_status mrcm_smooth(mrcm_ctx* ctx, int nsteps);

/* Execution of the smoothing sweeps (Steps 6-7).  use_graph != 0 (default):
 * the nsteps sweeps of an mrcm_smooth call (nsteps x 2^dim colour phases)
 * are captured into one HIP graph at the first call with that step count
 * after a configuration change, and replayed as one launch on the context's
 * stream.  threads_per_box: 64, 128 or 256 threads per
 * oversampled box, or 0 (default) to time the three on one sweep over a copy
 * of the current state and keep the fastest (done once per configuration,
 * outside the timed region of mrcm_smooth).  The choice does not change the
 * results.  3-D boxes take one to four waves by their plane size and ignore
 * threads_per_box; in the FP32 form the autotuner instead times how many
 * planes' inverses a box holds in registers (mrcm_stats.smooth_cached).
 * Errors: MRCM_EINVAL. */
mrcm_status mrcm_set_smoothing(mrcm_ctx* ctx, int use_graph, int threads_per_box);

/* Persistent form of the smoothing sweeps (Steps 6-7, Algorithm 1's loop
 * over the colours).  on != 0: each mrcm_smooth runs all its colour phases
 * in ONE cooperative launch; the workgroups (as many as the device holds at
 * once, at most max_groups when max_groups > 0, never more than the boxes of
 * the largest colour) loop over the boxes of a colour and meet at a
 * device-wide barrier between colours, which removes the launch gaps
 * between phases.  Applies to MRCM_FP64 contexts using the wave-per-box
 * kernels (2-D boxes, lines of at most 32 cells) without checkpointing;
 * otherwise, or when the device has no cooperative launch, mrcm_smooth uses
 * the per-phase launches of mrcm_set_smoothing.  The threads per box are the
 * ones mrcm_set_smoothing selects.  Results are bit-identical to the
 * per-phase form.  Default: off.  Errors: MRCM_EINVAL (max_groups < 0). */
mrcm_status mrcm_set_smoothing_persistent(mrcm_ctx* ctx, int on, int max_groups);

/* Tolerance of the interface solve's check (default 1e-5): the largest
 * componentwise backward error of the interface equations that
 * mrcm_solve_interface accepts (mrcm_stats.interface_residual); above it the
 * solve reports MRCM_ESINGULAR.  The block cyclic reduction does not pivot,
 * and on very ill-conditioned interface systems (Robin parameters far above
 * one) it can exceed the tolerance where the pivoted banded LU
 * (MRCM_IFACE_BAND_LU) does not.  tol <= 0 turns the check off (the
 * residual is still measured).  Errors: MRCM_EINVAL (NaN). */
mrcm_status mrcm_set_interface_check(mrcm_ctx* ctx, double tol);

/* Phase timing (default on): HIP events on the context's stream around the
 * phases of mrcm_build_basis, mrcm_solve_interface and mrcm_smooth, read by
 * mrcm_get_stats (ms_basis, ms_basis_kernel, ms_interface,
 * ms_interface_solve, ms_smooth of the last such call made with timing on).
 * Off, the calls enqueue their kernels only.  Results are unchanged.
 * Errors: MRCM_EINVAL (ctx NULL). */
mrcm_status mrcm_set_timing(mrcm_ctx* ctx, int on);

/* Deferred errors (default off), for callers that keep several contexts
 * busy at once, each on its own stream (a batch of independent problems).
 * Off, every call that produces results (mrcm_get_pressure, mrcm_get_flux,
 * mrcm_get_solution, mrcm_adjoint) ends by reading the device error flags,
 * which synchronises the context's stream.  On, those calls only enqueue
 * their work and return MRCM_OK; the flags stay set on the device across
 * calls (mrcm_build_basis no longer clears them) until mrcm_wait reads them.
 * Results written since the last mrcm_wait are valid only if it returns
 * MRCM_OK.  Switching off reads the flags as mrcm_wait does and returns its
 * status.  Host-side argument and state errors are still returned at once.
 * Errors: MRCM_EINVAL (ctx NULL). */
mrcm_status mrcm_set_deferred_errors(mrcm_ctx* ctx, int on);

/* Waits for the work enqueued on the context's stream, then reads and clears
 * the device error flags: MRCM_OK, or the device-side error of any call made
 * since the last read (MRCM_EINVAL for a non-finite or non-positive
 * permeability, MRCM_ENOTPD, MRCM_ESINGULAR, MRCM_ENOCONV), with
 * mrcm_last_error describing it.  Works in either error mode. */
mrcm_status mrcm_wait(mrcm_ctx* ctx);

/* Pressure per cell (N values); shifted to zero mean when no side carries a
 * pressure condition. */
mrcm_status mrcm_get_pressure(mrcm_ctx* ctx, double* p_dev);

/* Outward normal velocity on every face of every cell, N x 2*dim values,
 * cell-major (face order -x, +x, -y, +y, -z, +z).  A face on the skeleton
 * carries the value of the subdomain owning the cell (the normal flux is
 * double-valued there). */
mrcm_status mrcm_get_flux(mrcm_ctx* ctx, double* flux_dev);

/* Pressure (as mrcm_get_pressure) and face velocities (as mrcm_get_flux) in
 * one call: both outputs are enqueued before the error flags of the solve
 * are read, so the stream is synchronised once.  Errors: MRCM_EINVAL (NULL
 * output), MRCM_ESTATE, and the errors of the solve that produced them. */
mrcm_status mrcm_get_solution(mrcm_ctx* ctx, double* p_dev, double* flux_dev);

/* Interface unknowns X (n_unknowns values, subdomain-major, seeds of each
 * subdomain in side order), device pointer.  For tests. */
mrcm_status mrcm_get_coefficients(mrcm_ctx* ctx, double* x_dev);

/* Reverse mode (gradient of a function of the outputs with respect to
 * log K).  mrcm_set_checkpointing(ctx, 1) before the mrcm_smooth calls makes
 * them keep the state (pressure and Gamma fluxes) before every colour phase
 * (device memory: one copy of both per phase; smoothing then runs as plain
 * launches).  Default off. */
mrcm_status mrcm_set_checkpointing(mrcm_ctx* ctx, int on);

/* dJ/dlog K (N values) of J(pressure, flux) at the current solution, given
 * dJdp = dJ/d(mrcm_get_pressure output) (N values, or NULL for zero) and
 * dJdflux = dJ/d(mrcm_get_flux output) (N x 2*dim values, or NULL).  The
 * vector-Jacobian product of the whole discrete map (basis, particular
 * problems, interface system, MRCM-O assembly, smoothing sweeps, outputs),
 * computed on the device by the reverse of each step: adjoint local solves
 * with the cached factors (the local matrices are symmetric), the
 * transposed interface system by the same cyclic reduction, the smoothing
 * phases in reverse order recomputed from the checkpoints.  The local
 * solves take the precision of the forward solve: with MRCM_FP32_REFINE,
 * the cached FP32 factors refined in FP64 to the same tolerance (and the
 * same iteration limit, MRCM_ENOCONV when it is reached), every forward box
 * solution recomputed by the forward pass's own refinement; the interface
 * system stays FP64.  Device pointers.
 * Requirements: 2-D boxes whose lines have <= 32 cells, the block cyclic
 * reduction interface solver, equal Robin parameters in both stages,
 * checkpointing on for every smoothing step since the last
 * mrcm_solve_interface.  Errors: MRCM_EINVAL, MRCM_ESTATE, MRCM_ENOCONV,
 * MRCM_EDEVICE. */
mrcm_status mrcm_adjoint(mrcm_ctx* ctx, const double* dJdp_dev, const double* dJdflux_dev,
                         double* dJdlogK_dev);

mrcm_status mrcm_get_stats(mrcm_ctx* ctx, mrcm_stats* out);

/* Device reductions of the current solution (after mrcm_solve_interface or
 * mrcm_smooth): the per-cell mass-balance residual r_c = sum_faces |e| u_e -
 * f_c h^d into cell_residual_dev (N values, device, or NULL), the jump
 * moments of every interface equation row into jumps_dev (n_unknowns values,
 * device, or NULL; row order of the interface system: per interface
 * Gamma_ij, i < j, in order of i then axis, its p flux rows
 * sum_e |e| mu (u_i + u_j) then its p pressure rows sum_e |e| mu (pi_i - pi_j)),
 * and the summary into *out (host).  Deterministic (fixed reduction order).
 * Synchronises the context's stream.  Errors: MRCM_EINVAL, MRCM_ESTATE,
 * MRCM_EDEVICE and the device errors of the solve. */
mrcm_status mrcm_get_balance(mrcm_ctx* ctx, double* cell_residual_dev, double* jumps_dev,
                             mrcm_balance* out);

/* mrcm_get_balance for callers that cannot allocate device memory (code
 * between HIP graph captures, tight serving loops, harnesses that forbid
 * hipMalloc): the same results, bit for bit, with the partial sums and
 * maxima in a static device array of 65536 doubles instead of the
 * context's workspace; the call makes no allocation of any kind.  Limit:
 * grids of at most 1,863,424 cells (MRCM_EINVAL beyond).  The array is one
 * per GPU, shared by every context on it and kept until the process ends:
 * calls that overlap in time on one GPU (on different streams or threads)
 * race on it and must be serialised by the caller.  Synchronises the
 * context's stream.  Errors: as mrcm_get_balance. */
mrcm_status mrcm_get_balance_static(mrcm_ctx* ctx, double* cell_residual_dev, double* jumps_dev,
                                    mrcm_balance* out);

/* Relative L2 distances of the current outputs (pressure as mrcm_get_pressure,
 * face velocities as mrcm_get_flux) from reference arrays on the device:
 * out[0] = ||p - p_ref|| / ||p_ref|| (NaN when p_ref_dev is NULL), out[1] the
 * same for the N x 2d face velocities (NaN when flux_ref_dev is NULL); out is
 * host memory of two doubles.  Deterministic device reductions (the flux
 * norms of Section 5 over per-cell face values).  Synchronises the stream. */
mrcm_status mrcm_rel_error(mrcm_ctx* ctx, const double* p_ref_dev, const double* flux_ref_dev,
                           double* out);

/* Message of the last failure on this context (never NULL). */
const char* mrcm_last_error(const mrcm_ctx* ctx);

mrcm_status mrcm_destroy(mrcm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MRCM_H */
