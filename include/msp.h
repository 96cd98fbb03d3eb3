/*
 * msp.h -- C ABI of libmsp: the PCG state solve K(rho) u = f of SIMP
 * linear elasticity, preconditioned by the two-level overlapping additive
 * Schwarz method M_EH+Rot of Zambrano, Serrano, Lazarov and Galvis,
 * "Fast multiscale contrast independent preconditioners for linear elastic
 * topology optimization problems" (arXiv:2006.13387).
 *
 * All work runs on one AMD MI355X (gfx950) in hand-written HIP kernels.
 * Pointers marked _dev are device pointers (any HIP allocation, e.g. the
 * data_ptr() of a torch tensor); _host pointers are host memory.  Every
 * call enqueues on the caller's stream and returns after its results are
 * complete on that stream unless stated otherwise.
 *
 * Numbering (the same in every argument):
 *   node (i,j[,k])          id = i + (nx+1)*(j + (ny+1)*k)
 *   DOF c of node p         id = dim*p + c          (interleaved)
 *   element (i,j[,k])       id = i + nx*(j + ny*k)
 *
 * Status codes: 0 success, > 0 a warning with valid outputs, < 0 an error
 * that leaves every output untouched.  msp_last_error() gives the text.
 */
#ifndef MSP_H
#define MSP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MSP_OK = 0,
  MSP_NOT_CONVERGED = 1,   /* maxit reached: u holds the last iterate     */
  MSP_E_INVALID = -1,      /* bad argument or unsupported problem shape   */
  MSP_E_NOMEM = -2,        /* device allocation failed                   */
  MSP_E_DEVICE = -3,       /* a HIP call failed                          */
  MSP_E_NOT_SPD = -4,      /* a local or coarse pivot was not positive   */
  MSP_E_BREAKDOWN = -5,    /* p^T K p <= 0 or a non-finite CG scalar     */
  MSP_E_STATE = -7         /* call out of order (e.g. solve before rho)  */
} msp_status;

/*
 * Problem statement (paper Section 1: SIMP law and Navier-Cauchy problem;
 * Section 2: coarse blocks D_i and overlapping subdomains D'_i; Section 4.1:
 * heat eigenproblem and its automatic threshold; Section 4.2: rotations).
 *
 *  dim        2 (bilinear Q1, plane stress) or 3 (trilinear H8, isotropic;
 *             in 3D sub_mode must be 0 and eig_random 0; eig_kmax = 0
 *             gives the first level alone (the paper's one-level method),
 *             eig_kmax in 1..24 the coarse space with three rotations per
 *             coarse node (Section 4.2) when rot_enrich is set; a node
 *             must then be clamped in all three components or in none)
 *  nel        elements per axis (nel[2] ignored in 2D)
 *  h          element edge length
 *  E0, Emin   SIMP moduli: E_e = Emin + rho_e^penal (E0 - Emin), 0<Emin<=E0
 *  nu         Poisson ratio in (-1, 0.5)
 *  penal      SIMP exponent, >= 1
 *  sub_nel    coarse block edge S in elements per axis (must divide nel)
 *  overlap    delta: element layers added around each block (0 <= delta < S,
 *             and 2 delta <= S so that a node lies in at most four subdomains)
 *  sub_mode   0: subdomains are the blocks extended by delta (max-norm);
 *             1: subdomains are the coarse-vertex neighbourhoods of the
 *                coarse nodes that are not clamped (the paper's experiments)
 *  eig_tau    keep heat eigenvalues with lambda * H^2 < eig_tau, H = S*h
 *  eig_kmax   at most this many modes per neighbourhood (1..24)
 *  rot_enrich 1: add chi_l times the rotations (M_EH+Rot); 0: M_EH
 *  precision  0: FP64 local solves; 1: local inverses stored, applied and
 *             accumulated in FP32 inside the FP64 outer CG (flexible beta),
 *             except in subdomains whose amplification metric (see
 *             msp_solve_info.fp64_subdomains) shows stiff islands floating
 *             in soft material, which keep FP64 blocks
 *  eig_random 0: heat eigenpairs by shift-invert subspace iteration to
 *             convergence; M in 1..31: the randomized approximation of
 *             Section 3 (M_EH+Rot;Rand) from M zero-mean random forcings,
 *             their local solutions with A + 0.05/H^2 M and the constant
 *             function, by Rayleigh-Ritz on that space.  With coarse_kind
 *             1 or 2 (M in 1..29) it applies to the elasticity pencils
 *             instead (M_EE;Rand): M random forcings free of net force,
 *             their solutions with K + 0.05/H^2 M, the rigid-body motions
 *             added, one Rayleigh-Ritz step; the heat count stays exact
 *  eig_seed   seed of the randomized forcings (SplitMix64, counter-based)
 *  coarse_kind 0: the heat coarse space (M_EH, M_EH+Rot; Section 4);
 *             1: M_EE (Section 2.1, 2D only): per coarse neighbourhood the
 *                lowest eigenpairs of the local elasticity pencil
 *                -div sigma(psi) = lambda E psi times chi_l, 3 per
 *                high-stiffness region of the neighbourhood (the regions
 *                counted by the heat threshold; at most 24 modes a
 *                neighbourhood); 2: M_EE with twice as many modes.
 *                M_EE keeps its coarse operator dense (n x N_c), for the
 *                paper's small examples; batches and serving refuse it.
 */
typedef struct {
  int32_t dim;
  int32_t nel[3];
  double h, E0, Emin, nu, penal;
  int32_t sub_nel[3];
  int32_t overlap;
  int32_t sub_mode;
  double eig_tau;
  int32_t eig_kmax;
  int32_t rot_enrich;
  int32_t precision;
  int32_t eig_random;
  uint32_t eig_seed;
  int32_t coarse_kind;
} msp_problem_desc;

typedef struct {
  int32_t status;          /* msp_status of the solve                        */
  int32_t iters;           /* PCG iterations (all restarts included)         */
  int32_t converged;       /* 1 if the true residual met rtol                */
  int32_t restarts;        /* restarts from the true residual                */
  int32_t n_coarse;        /* coarse dimension N_c (columns of R_0^T)         */
  int32_t coarse_rank;     /* numerical rank of K_0                          */
  int32_t cap_hits;        /* neighbourhoods with more than kmax modes below  */
  int32_t fp64_subdomains; /* subdomains applied with FP64 inverse blocks     */
  int32_t eig_unconverged; /* neighbourhoods whose heat eigen iteration hit
                              its step limit before the Ritz values deciding
                              the threshold settled (0 on a sound setup)     */
  int32_t setup_reused;    /* 1: this solve ran with a setup built for
                              earlier densities (lazy reuse, serving)       */
  double relres_true;      /* ||f - K u|| / ||f|| over free DOFs             */
  double relres_rec;       /* recursively updated residual at exit           */
  double compliance;       /* f^T u                                          */
  double cond_est;         /* Lanczos estimate of cond(M^-1 K) (Section 5)   */
  double t_setup_ms;       /* setup run inside this call (0 if none)         */
  double t_solve_ms;       /* PCG wall time of this call                     */
} msp_solve_info;

typedef struct msp_handle msp_handle;

/*
 * Create a solver for one mesh.  fixed_mask_host holds n = dim*(#nodes)
 * bytes, 1 = that displacement DOF is clamped to zero (Gamma_D).  The mask
 * is copied.  In 2D the block row of a subdomain (2 * nodes per row) and
 * of a neighbourhood (nodes per row) must not exceed 72.  A 3D handle
 * supports every single-problem call: a subdomain may hold at most 2,048
 * DOFs (7^3 nodes for S = 6 and one overlap layer) and a neighbourhood's
 * node plane (constant z) at most 256 nodes (S <= 7 in x and y); the
 * geometry is checked by the first msp_setup.  Batches and serving return
 * MSP_E_INVALID for a 3D handle; without a coarse space msp_apply_coarse
 * gives z = 0.
 * Errors: MSP_E_INVALID (see the field ranges above), MSP_E_NOMEM.
 */
msp_status msp_create(const msp_problem_desc* desc,
                      const uint8_t* fixed_mask_host, msp_handle** out);

/* Free every device buffer of the handle.  Accepts NULL. */
msp_status msp_destroy(msp_handle* h);

/* Text of the last error on this handle (static storage if h is NULL). */
const char* msp_last_error(const msp_handle* h);

/*
 * Element densities rho_dev (nel doubles in [0,1]) for the next setup.
 * Computes E_e by the SIMP law on the device and marks the setup dirty.
 * Non-finite or out-of-range densities give MSP_E_INVALID.
 */
msp_status msp_set_densities(msp_handle* h, const double* rho_dev,
                             hipStream_t stream);

/*
 * Build the preconditioner for the current densities (Section 2 and 4):
 * local factors of K_i = R_i K R_i^T, heat eigenpairs on every coarse
 * neighbourhood with the threshold, coarse basis and K_0^+.  One
 * device-to-host read of the selected mode counts.  MSP_E_NOT_SPD if a
 * local pivot is not positive.  3D: the dense inverse of every K_i
 * (FP64, and an FP32 copy when precision = 1), held by the handle
 * (about 12 ld^2 bytes per subdomain, ld the largest local order rounded
 * up to 64); with eig_kmax > 0 the heat pencils of all coarse
 * neighbourhoods factored by node planes (8 ldp^2 bytes a plane, ldp the
 * largest plane rounded up to 64) and solved by subspace iteration, and
 * K_0 held as block LDL^T factors by slabs of coarse nodes (columns
 * that are linearly dependent by construction, one rotation per plane of
 * coarse nodes that all carry rotations, are dropped).  MSP_E_INVALID if
 * the subdomains or planes are too large, the subdomains do not cover the
 * free DOFs, a node is clamped in only some components, or N_c exceeds
 * 32,768.
 */
msp_status msp_setup(msp_handle* h, hipStream_t stream);

/*
 * Solve K_FF u = f by PCG with M_EH+Rot (M_EH; the first level alone when
 * eig_kmax = 0 in 3D) to
 * ||f - K u|| <= rtol ||f|| over the free DOFs (Section 2; Section 5 for the stopping
 * test and the Lanczos estimate).  f_dev and u_dev hold nrhs right-hand
 * sides of n doubles each, one after another; with warm != 0 u_dev holds
 * the initial guesses.  Entries of f at clamped DOFs are ignored and u is
 * 0 there.  Runs msp_setup first if the densities changed.  info_host (may
 * be NULL) receives the statistics of the last right-hand side.
 */
msp_status msp_solve(msp_handle* h, const double* f_dev, double* u_dev,
                     int32_t nrhs, int32_t warm, double rtol, int32_t maxit,
                     hipStream_t stream, msp_solve_info* info_host);

/*
 * Lazy reuse of the preconditioner across density updates (Section 1: the
 * preconditioner is updated after a fixed number of optimisation steps, or
 * once the iterations of the solver exceed a threshold).  With max_age > 0
 * a setup built for earlier densities is kept for up to max_age further
 * msp_set_densities calls: msp_solve (and the single-step applies, batches
 * and serving) then run PCG on the new K(rho) preconditioned by the older
 * setup, which is still symmetric positive definite, so the solution is
 * that of the new system to rtol.  With iter_limit > 0, msp_solve stops a
 * solve on a reused setup after iter_limit iterations, rebuilds the setup
 * for the current densities and continues from the iterate it reached
 * (msp_solve_info.iters counts both parts; batches and serving instead make
 * the next solve rebuild).  max_age = 0 (the default) rebuilds at every
 * density change.  msp_solve_info.setup_reused tells which solves finished
 * on an older setup.
 * Errors: MSP_E_INVALID for negative arguments.
 */
msp_status msp_set_reuse(msp_handle* h, int32_t max_age, int32_t iter_limit);

/* ---- single steps of the hot path, for parity checks and profiling ---- */

/* y = K_FF x (Section 1.1 discretisation, Q1 plane stress in 2D, H8 in
 * 3D): y = 0 at clamped DOFs, entries of x at clamped DOFs are treated as
 * 0.  x and y are device vectors of n = dim * #nodes doubles (interleaved
 * DOFs) that must not alias.  Needs densities. */
msp_status msp_apply_K(msp_handle* h, const double* x_dev, double* y_dev,
                       hipStream_t stream);

/* z = sum_i R_i^T K_i^{-1} R_i r  (first level, Section 2).  Needs setup. */
msp_status msp_apply_level1(msp_handle* h, const double* r_dev, double* z_dev,
                            hipStream_t stream);

/* z = R_0^T K_0^+ R_0 r  (coarse level, Sections 2 and 4.3). */
msp_status msp_apply_coarse(msp_handle* h, const double* r_dev, double* z_dev,
                            hipStream_t stream);

/* z = M^{-1} r = level 1 + coarse level. */
msp_status msp_apply_prec(msp_handle* h, const double* r_dev, double* z_dev,
                          hipStream_t stream);

/*
 * Coarse-space statistics after setup.  n_modes_host: one int per coarse
 * node (x fastest) = heat modes selected; eigvals_host: eig_kmax doubles
 * per coarse node (selected eigenvalues ascending, rest NaN).  Either
 * pointer may be NULL.  n_coarse_nodes receives the coarse node count.
 */
msp_status msp_coarse_info(msp_handle* h, int32_t* n_modes_host,
                           double* eigvals_host, int32_t* n_coarse_nodes,
                           int32_t* n_coarse, int32_t* cap_hits);

/* Write the coarse basis R_0^T as a dense n x N_c column-major matrix to
 * phi_dev (caller allocates n*N_c doubles).  For checks on small meshes. */
msp_status msp_coarse_basis(msp_handle* h, double* phi_dev, hipStream_t stream);

/* Write a coarse matrix to out_dev (caller allocates ldk * ldk doubles,
 * ldk = msp_query()[11]; row-major with leading dimension ldk, entries
 * beyond N_c are padding): which = 0 the assembled K_0 = R_0 K R_0^T of the
 * last setup (Section 2; recomputed from the stored K R_0^T columns),
 * which = 1 the generalised inverse K_0^+ that the coarse solve applies
 * (2D only: a 3D handle keeps K_0 as slab factors and returns
 * MSP_E_INVALID).  For checks of the coarse solve.  Errors: MSP_E_INVALID,
 * MSP_E_STATE (no setup, or no coarse space), MSP_E_DEVICE. */
msp_status msp_coarse_matrix(msp_handle* h, int32_t which, double* out_dev,
                             hipStream_t stream);

/* out_host[0] = x . y over n doubles with the library's two-stage
 * wavefront reduction (the reduction used by the CG dot products). */
msp_status msp_vec_dot(int64_t n, const double* x_dev, const double* y_dev,
                       hipStream_t stream, double* out_host);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid hipMalloc): out_dev[0] = x . y over n
 * doubles, the same kernel and grid as msp_vec_dot (so the same bits), but
 * with its workgroup partials and ticket counter in a fixed library-owned
 * device array (1,025 doubles per GPU, held until the process ends) instead
 * of buffers allocated per call, and the result left in device memory
 * (out_dev: one double, caller-owned).  Nothing is allocated and the call
 * does not synchronise: the result is ready when the caller's stream
 * reaches it.  Every call on a GPU shares that GPU's array, so calls that
 * overlap on one GPU (different streams, or host threads) race; serialise
 * them.  The first call on each device looks the array up (with that
 * device current).
 * Errors: MSP_E_INVALID (null pointer, n < 0, n > MSP_NOALLOC_DOT_MAX_N),
 * MSP_E_DEVICE.  The text is in msp_last_error(NULL).
 */
#define MSP_NOALLOC_DOT_MAX_N (((int64_t)1) << 35)
msp_status msp_vec_dot_noalloc(int64_t n, const double* x_dev,
                               const double* y_dev, double* out_dev,
                               hipStream_t stream);

/* Sizes (12 int64): [0] n DOFs, [1] elements, [2] subdomains, [3] coarse
 * nodes, [4] coarse dimension after setup, [5] largest local system,
 * [6] bytes of first-level factor records (inverse Schur blocks and row
 * couplings, in the precision selected per subdomain) that one first-level
 * application reads, [7] bytes of stored heat modes psi,
 * [8] sum of local system sizes, [9] sum of neighbourhood sizes,
 * [10] bytes of the neighbourhood inverse blocks, [11] padded K_0 order. */
msp_status msp_query(msp_handle* h, int64_t* sizes12);

/*
 * Per-kernel event timing for measurement.  enable >= 0 is a bit mask of
 * the tracked kernels below: from now on the library records a hipEvent
 * pair around every launch of each selected kernel on the caller's stream
 * (0 stops timing, -1 leaves the state unchanged).
 * Before changing the state the call returns, for kernel k < n, the number
 * of timed launches and their summed duration in ms since the last reset:
 * k = 0 first-level apply, 1 stiffness product (in the CG and in
 * msp_apply_K), 2 heat eigen setup,
 * 3 combine (z = M^-1 r), 4 coarse restriction, 5 local factorisation.
 */
msp_status msp_kernel_timing(msp_handle* h, int32_t enable,
                             int64_t* launches_host, double* total_ms_host,
                             int32_t n);

/* ---- the design update around the state solve (Section 1) ---- */

/*
 * Gradient of an objective with respect to the element densities,
 * Section 1's formula d g/d rho_e = -u^T (dK/d rho_e) u for the compliance
 * f^T u, under the SIMP law of the handle:
 *   dg_dev[e] = -p rho_e^(p-1) (E0 - Emin) lam_e^T K^_e u_e
 * (K^_e the unit-modulus element matrix, u_e / lam_e the element's DOFs).
 * lam_dev = NULL means lam = u (compliance); otherwise lam is the adjoint
 * solution of K lam = l for an objective l^T u.  rho_dev, dg_dev: nel
 * doubles; u_dev, lam_dev: n doubles.  2D and 3D handles.  dg_dev must not
 * alias an input.  Errors: MSP_E_INVALID, MSP_E_DEVICE.
 */
msp_status msp_sensitivity(msp_handle* h, const double* rho_dev,
                           const double* u_dev, const double* lam_dev,
                           double* dg_dev, hipStream_t stream);

/*
 * One optimality-criteria density update (the method Section 1 names for
 * the design step, after Bendsoe and Sigmund): with B_e = max(0, -dg_e)/Lam,
 *   rho_new[e] = clamp(rho_e sqrt(B_e), max(0, rho_e - move),
 *                      min(1, rho_e + move)),
 * the multiplier Lam chosen on the device (a logarithmic bracketing pass,
 * then passes that split the bracket 33-fold, to a relative width of
 * 1e-13) so that sum_e rho_new[e] = volfrac * nel (equal element volumes).
 * If even Lam = 2^75 leaves the volume above the target, Lam = 2^75.  No
 * density filter.  rho_dev, dg_dev, rho_new_dev: nel doubles (rho_new_dev
 * must not alias the inputs); *lam_host receives Lam (may be NULL).
 * Errors: MSP_E_INVALID (volfrac or move outside (0, 1]), MSP_E_NOMEM,
 * MSP_E_DEVICE, MSP_E_BREAKDOWN (the search did not converge).
 */
msp_status msp_oc_update(msp_handle* h, const double* rho_dev,
                         const double* dg_dev, double volfrac, double move,
                         double* rho_new_dev, double* lam_host,
                         hipStream_t stream);

/* ---- batches: the PCG solves of many problems in lockstep ---- */

typedef struct msp_batch msp_batch;

/* Create / destroy a batch context (device tables and a captured graph,
 * reused while the same handles are solved together). */
msp_status msp_batch_create(msp_batch** out);
msp_status msp_batch_destroy(msp_batch* b);
const char* msp_batch_last_error(const msp_batch* b);

/*
 * Solve problem e = 0..n-1 on its own handle hs[e] (all distinct, densities
 * set): K_e u_e = f_e to rtol as msp_solve does, with warm[e] (may be NULL)
 * selecting a warm start from u_e.  Setups run first where the densities
 * changed.  Every PCG iteration then launches each iteration kernel once
 * for all problems still iterating (the first-level solves of all of them
 * in one persistent launch of one workgroup per CU); with use_graph != 0 a
 * chunk of iterations is captured once as a HIP graph and replayed.  The
 * launch shape (iterations per chunk: 8, 16 or 32; the first-level items
 * problem by problem or largest systems first) is picked by an autotuner:
 * the first chunks run on a new set of handles measure each candidate
 * twice, in a mirrored order, as wall time per iteration per active DOF
 * (carried over to the next solves until complete), and the fastest is
 * kept for that set.  Each problem's arithmetic is that of msp_solve on its
 * handle whatever the shape, so every result is bitwise the one it would
 * have alone.  infos_host (may be NULL)
 * receives n statistics records.  A negative status of any entry makes the
 * call return an error; MSP_NOT_CONVERGED if some entry did not converge.
 */
msp_status msp_batch_solve(msp_batch* b, msp_handle* const* handles,
                           const double* const* f_dev, double* const* u_dev,
                           const int32_t* warm_host, int32_t n, double rtol,
                           int32_t maxit, int32_t use_graph, hipStream_t stream,
                           msp_solve_info* infos_host);

/* Chunks of lockstep iterations run by this batch context, and how many
 * of them were graph replays. */
msp_status msp_batch_stats(const msp_batch* b, int64_t* chunks,
                           int64_t* graph_chunks);

/* Switch the launch-shape autotuner on (default) or off (off: 16 iterations
 * per chunk, items problem by problem). */
msp_status msp_batch_set_autotune(msp_batch* b, int32_t on);

/* The current launch shape (chunk: iterations per chunk; order: 1 when the
 * first-level items go largest systems first), whether it is the tuned
 * choice for the last set of handles (tuned = 1), and the measured cost of
 * each of the 6 candidates (ms per iteration per active DOF; 0: not yet
 * measured), candidates in the order (16, 8, 32 iterations) x (problem
 * order, largest first).  cost_host may be NULL. */
msp_status msp_batch_tuning(const msp_batch* b, int32_t* chunk, int32_t* order,
                            int32_t* tuned, double* cost_host);

/* ---- serving: continuous batching of state and adjoint solves ---- */

typedef struct msp_server msp_server;

/*
 * A request loop for many topology-optimisation runs.  A run is a mesh with
 * its clamped DOFs (2D, or 3D with the heat coarse space); its handle
 * (setup) and its last state and adjoint solutions stay resident while the
 * projected device memory of all resident runs fits hbm_budget_bytes (idle
 * runs' setups are evicted least recently used first; their warm-start
 * vectors stay).  A run's projection is raised to the device bytes its
 * handle was measured to hold once admitted.  At most max_active requests
 * are in progress.  The serving layer is not in the paper; the solves are.
 */
msp_status msp_server_create(int64_t hbm_budget_bytes, int32_t max_active,
                             msp_server** out);
msp_status msp_server_destroy(msp_server* sv);
const char* msp_server_last_error(const msp_server* sv);

/* Register a run (validated like msp_create and, in 3D, like msp_setup's
 * buffer layout; no device memory is kept). */
msp_status msp_server_add_run(msp_server* sv, const msp_problem_desc* desc,
                              const uint8_t* fixed_mask_host, int32_t* run_id);

/*
 * Queue a request of a run: new densities, a state load and optionally an
 * adjoint load (f_adj_dev and u_adj_dev both NULL for none).  The solutions
 * are written to u_state_dev / u_adj_dev when the request completes; each
 * solve warm-starts from the run's previous solution of its kind.  The
 * caller keeps all five device arrays alive until then.  Requests of one
 * run are served in submission order.
 */
msp_status msp_server_submit(msp_server* sv, int32_t run_id,
                             const double* rho_dev, const double* f_state_dev,
                             const double* f_adj_dev, double* u_state_dev,
                             double* u_adj_dev, double rtol, int32_t maxit,
                             int32_t* ticket);

/*
 * One scheduling step on the caller's stream: one chunk of 16 lockstep PCG
 * iterations for every 2D solve in progress (a batched launch per iteration
 * kernel, as msp_batch_solve) and 16 iterations of each 3D solve in
 * progress, while queued requests are admitted as slots
 * and memory allow, their densities and setup running on a second stream
 * at the same time (ordered after all work the caller queued on the stream
 * before this call, so densities written there are seen); then finished
 * solves move on (state -> adjoint -> done).  n_completed receives the requests completed by this step.  Each
 * solve's arithmetic is that of msp_solve on its run's handle with the
 * same warm start, whatever else is in progress.
 */
msp_status msp_server_step(msp_server* sv, hipStream_t stream,
                           int32_t* n_completed);

/* Result of a completed request: two msp_solve_info records (state,
 * adjoint) and the latency from submission to completion in ms.
 * MSP_E_STATE while the request is still queued or in progress. */
msp_status msp_server_result(msp_server* sv, int32_t ticket,
                             msp_solve_info* info2_host, double* latency_ms);

/* Lazy preconditioner reuse for every run of the server (msp_set_reuse's
 * policy, applied to each run's handle; a run whose setup was evicted
 * rebuilds).  The decision is taken when a request is admitted: its state
 * and adjoint solves share one setup. */
msp_status msp_server_set_reuse(msp_server* sv, int32_t max_age,
                                int32_t iter_limit);

/* Writes min(n, 10) doubles: completed requests, p50 and p99 latency (ms),
 * solves per second (state and adjoint solves, first submission to last
 * completion), projected device bytes of resident runs, queued, active,
 * chunks run, setups built, setups reused. */
msp_status msp_server_stats(const msp_server* sv, double* stats_host, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* MSP_H */
