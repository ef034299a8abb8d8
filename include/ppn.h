/*
 * ppn.h -- C ABI of the MI355X (gfx950) implementation of Progressively
 * Projected Newton (PPN) for implicit hyperelastic time stepping on linear
 * tetrahedra, with Projected Newton (PN) and Project-on-Demand Newton (PDN)
 * as comparison modes (arXiv 2505.21013).
 *
 * One time step is the minimisation of the backward-Euler incremental
 * potential (Sec. 3, Eq. (1); Sec. 5.1 "Time stepping and tolerances")
 *     Psi(x) = sum_i m_i/(2h^2)|x_i - xhat_i|^2 + sum_e V_e psi(F_e)
 *              + sum_{i in D} k_D/2 |x_i - xbar_i|^2
 * by Newton's method, where psi is the Stable Neo-Hookean energy
 *     psi(F) = mu/2 (tr F^T F - 3) - mu (J - 1) + lam/2 (J - 1)^2
 * with mu = mu_L, lam = lam_L + mu_L from (E, nu) (Sec. 5.1, material model),
 * lumped masses m_i = sum_{e ni i} rho V_e/4, xhat = x^n + h v^n + h^2 g_grav
 * and Dirichlet constraints as penalty potentials (Sec. 5.1).
 *
 * Conventions for every entry point:
 *  - Pointers are HOST memory unless the parameter name ends in "_dev".
 *    Inputs are copied during the call; the caller keeps ownership.
 *  - The library owns all of its device memory (hipMalloc at load time).
 *  - Vectors of points are AoS, [n][3] doubles (x0 y0 z0 x1 ...).
 *  - Every function returns a ppn_status: negative = error, nothing changed;
 *    positive = warning, the state did advance.  No exception crosses the
 *    ABI; ppn_last_error() gives the message of the last failing call.
 *  - A scene handle is used by one host thread at a time and is bound to the
 *    HIP stream given at creation (NULL = a stream the library creates).
 *    Calls are synchronous with respect to that stream: on return, results
 *    are final.
 */
#ifndef PPN_H
#define PPN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ppn_scene ppn_scene; /* opaque, library-owned */

/* Newton variants.  PN: project every element Hessian (Sec. 3).  PDN: project
 * all elements once indefiniteness is detected, then for a countdown of
 * iterations (Sec. 2.2, Sec. 5.1).  PPN: Algorithm 1 (Sec. 4). */
typedef enum { PPN_PN = 0, PPN_PDN = 1, PPN_PPN = 2 } ppn_mode;

/* Arithmetic of the hot path.  PPN_FP64: everything in FP64.  PPN_MIXED:
 * eigensolves in FP32; inside PCG the assembled matrix and block-Jacobi
 * inverse are stored in FP32 and the matrix product is formed and accumulated
 * in FP32, while the CG vectors, their recurrences and all dot products stay
 * FP64; element energies, gradients, Hessian assembly, the Newton residual,
 * the line-search energy sum and the iterative-refinement residual of each
 * linear solve stay FP64 (the solve is repeated on the FP64 residual until
 * that meets pcg_rtol). */
typedef enum { PPN_FP64 = 0, PPN_MIXED = 1 } ppn_precision;

/* Newton stopping rule.  VEL (Sec. 5.1): stop once |dx|_inf / h < stop_tol
 * after the solve, without applying that step.  GRAD_REL: stop at the top of
 * iteration k once |g^k|_2 <= stop_tol |g^0|_2. */
typedef enum { PPN_STOP_VEL = 0, PPN_STOP_GRAD_REL = 1 } ppn_stop_mode;

typedef enum {
  PPN_OK = 0,
  PPN_ERR_ARG = -1,    /* invalid argument or call order */
  PPN_ERR_MESH = -2,   /* invalid mesh (see ppn_load_mesh), or a rest tet with det(Dm) <= 0 */
  PPN_ERR_OOM = -3,    /* device allocation failed */
  PPN_ERR_DEVICE = -4, /* a HIP call failed (message in ppn_last_error) */
  PPN_ERR_STATE = -5,  /* non-finite positions or velocities */
  PPN_WARN_NOT_CONVERGED = 1, /* newton_maxit reached; the step was taken */
  PPN_WARN_LS_FAIL = 2        /* no Armijo step within ls_maxit halvings */
} ppn_status;

/* Solver parameters.  Defaults (ppn_params_default) follow the paper:
 * alpha 0.5, beta 2, eps_delta 1e-12 (Sec. 4); eps_clamp 1e-8, PCG relative
 * tolerance 1e-4, PDN countdown 4, velocity tolerance 1e-3 m/s (Sec. 5.1).
 * The remaining values are readings: pcg_maxit 10000, newton_maxit 100,
 * Armijo c 1e-4 with at most 30 halvings, k_dirichlet 1e8 N/m; use_graphs 1. */
typedef struct {
  double alpha;         /* tightening factor, 0 < alpha < 1 */
  double beta;          /* release factor, >= 1 */
  double eps_delta;     /* PN fallback threshold on delta */
  double eps_clamp;     /* eigenvalue clamp eps > 0 */
  double pcg_rtol;      /* |r|/|r0| */
  int32_t pcg_maxit;
  int32_t pdn_countdown;
  int32_t stop_mode;    /* ppn_stop_mode */
  int32_t newton_maxit;
  double stop_tol;
  double armijo_c;
  int32_t ls_maxit;
  int32_t eig_mirror;    /* 0: clamp eigenvalues to max(lambda, eps) (Eq. (4)); 1: mirror them,
                            max(|lambda|, eps) (the alternative filter of Sec. 2 and Sec. 5) */
  double k_dirichlet;   /* penalty stiffness [N/m] */
  int32_t pcg_load_mode; /* -1 (default): chosen from the matrix size (0 up to 64 MB of values,
                            else 1); 0 small, 1 ordinary loads with capped residency, 2 streamed
                            with non-temporal loads: forces how the PCG product of this scene's own
                            solves loads the matrix.  Every mode gives the same bits; for tuning and
                            tests.  Batched engine launches always choose from the summed size. */
  int32_t use_graphs;    /* 1 (default): a scene stepped alone runs the kernels of each Newton
                            iteration's evaluation (element quantities, assembly, gradient
                            norms) as one HIP graph captured at its first use; 0: plain
                            launches.  The same kernels either way, so the same bits. */
} ppn_params;

/* Statistics of one time step. */
typedef struct {
  int32_t newton_iters;      /* Newton iterations entered (gradient evaluations) */
  int32_t pcg_iters;         /* products H d over all solves */
  int32_t solves;            /* PCG solves actually run */
  int32_t indefinite_solves; /* solves that reported indefiniteness */
  int32_t inner_rounds;      /* PPN selection rounds (Algorithm 1 inner loop) */
  int32_t ls_backtracks;     /* line-search halvings */
  int32_t safety_events;     /* solves still indefinite with every element projected */
  int32_t converged;         /* 1 if the stopping rule was met */
  int32_t ls_fail;           /* 1 if the line search failed */
  int32_t skipped_solves;    /* PPN rounds that projected nothing new, so the unchanged
                                system was not solved again (its result is known) */
  int64_t projected;         /* element Hessians eigendecomposed, summed over iterations */
  double res0_l2;            /* |g|_2 at the first iterate of the step */
  double res_l2;             /* |g|_2 at the last evaluated iterate */
  double res_inf;            /* |g|_inf at the last evaluated iterate */
  double ms_total;           /* wall time of the step [ms] */
  double ms_eig;             /* time in the eigen-projection kernel [ms] */
  double ms_pcg;             /* time in PCG solves [ms] */
  double ms_spmv;            /* summed duration of the sampled PCG matrix-product launches,
                                measured with HIP events when profiling is on (else 0) [ms] */
  int64_t n_spmv;            /* sampled launches summed in ms_spmv */
  int32_t refine_rounds;     /* PPN_MIXED: PCG runs with the FP32 matrix (each followed
                                by an FP64 residual); 0 in PPN_FP64 */
  int32_t reserved1;
} ppn_step_stats;

/* One record per Newton iteration of the last step (when tracing is on). */
typedef struct {
  int32_t k;            /* iteration index within the step */
  int32_t first_ind;    /* indefiniteness reported by the first solve */
  int32_t first_iters;  /* PCG iterations of the first solve */
  int32_t rounds;       /* PPN inner rounds */
  int32_t n_projected;  /* elements projected in this iteration */
  int32_t last_ind;     /* indefiniteness of the final solve */
  double g_l2, g_inf;   /* gradient norms at this iterate */
  double delta_in;      /* delta on entry (INFINITY if unset) */
  double delta_out;     /* delta after the relax step */
  double dx_inf;        /* |dx|_inf of the final direction */
  double gamma;         /* accepted line-search step (0 if none / converged) */
} ppn_iter_record;

/* Fill *out with the defaults above. */
ppn_status ppn_params_default(ppn_params* out);

/* Create an empty scene on the current HIP device.  hip_stream may be NULL
 * (the library creates a default-priority stream) or a hipStream_t of the
 * caller, which must outlive the scene. */
ppn_status ppn_scene_create(ppn_scene** out, void* hip_stream, int32_t precision);
ppn_status ppn_scene_destroy(ppn_scene* s);

/* Load a tetrahedral mesh: rest positions [n_verts][3], tets [n_tets][4]
 * (0-based, positively oriented: det[X1-X0, X2-X0, X3-X0] > 0), optional
 * initial positions (NULL = rest).  Builds the block-sparse pattern and the
 * element->slot maps, allocates device memory, computes Dm^-1, V_e and the
 * lumped masses (needs the material; default rho 1000, E 1e5, nu 0.45 until
 * ppn_set_material is called).  Velocities start at zero.  Errors:
 * PPN_ERR_MESH for an index out of range, a tet that repeats a vertex, a
 * vertex that belongs to no tet, det(Dm) <= 0, or a mesh beyond the 32-bit
 * index limits (at most 238,609,294 tets; at most 2^31 sliced-ELL block
 * positions, about 140M vertices of a regular tet grid); PPN_ERR_OOM when the
 * device memory does not hold it (about 1.2 KB per tet in PPN_FP64, so one
 * 288 GB GPU holds about 230M tets). */
ppn_status ppn_load_mesh(ppn_scene* s, int32_t n_verts, const double* rest_xyz,
                         int32_t n_tets, const int32_t* tets, const double* init_xyz);

/* Density [kg/m^3] and Young's modulus / Poisson ratio, either one value each
 * (per_element = 0) or one per tet (per_element = 1, arrays of n_tets), of the
 * Stable Neo-Hookean material (Sec. 5.1); recomputes the lumped masses.
 * PPN_ERR_ARG unless 0 <= nu < 0.5, E >= 0, rho > 0 (or per_element without
 * a loaded mesh); PPN_ERR_MESH if a rest tet has det(Dm) <= 0. */
ppn_status ppn_set_material(ppn_scene* s, double rho, const double* E, const double* nu,
                            int32_t per_element);

/* Time step h [s] of the backward-Euler potential (Sec. 3, Eq. (1)) and
 * gravity [3] (m/s^2; NULL keeps the current value).  PPN_ERR_ARG unless h is
 * finite and > 0. */
ppn_status ppn_set_time_step(ppn_scene* s, double dt, const double* gravity);

/* Dirichlet penalty set (Sec. 5.1, penalty potentials with stiffness
 * k_dirichlet): n vertex ids (any order, no duplicates) and their targets
 * [n][3] at the END of the next time step.  Replaces the previous set; call
 * again before each step to move the targets.  PPN_ERR_ARG for an id out of
 * range or repeated, a non-finite target, or no loaded mesh. */
ppn_status ppn_set_dirichlet(ppn_scene* s, int32_t n, const int32_t* vert_ids,
                             const double* target_xyz);

/* Parameters of Algorithm 1 and of the solvers (defaults: ppn_params_default).
 * PPN_ERR_ARG, with nothing changed, unless 0 < alpha < 1, beta >= 1,
 * eps_clamp > 0, eps_delta >= 0, 0 < pcg_rtol < 1, pcg_maxit >= 1, a known
 * stop_mode, stop_tol >= 0, newton_maxit >= 1, ls_maxit >= 0, pdn_countdown
 * >= 0, 0 < armijo_c < 1, k_dirichlet >= 0 and eig_mirror in {0, 1}. */
ppn_status ppn_set_params(ppn_scene* s, const ppn_params* p);

/* Advance one time step with the given Newton variant (Algorithm 1 for
 * PPN_PPN; Sec. 2.2 and Sec. 5.1 for PN and PDN).  out may be NULL.  Returns
 * PPN_OK; PPN_WARN_NOT_CONVERGED after newton_maxit iterations or
 * PPN_WARN_LS_FAIL when the line search fails (the state advanced up to that
 * iteration); PPN_ERR_ARG for an unknown mode or no mesh; PPN_ERR_STATE for a
 * non-finite gradient; PPN_ERR_DEVICE for a HIP failure. */
ppn_status ppn_newton_step(ppn_scene* s, int32_t mode, ppn_step_stats* out);

/* Current positions: host copy [n_verts][3], or device-to-device copy into a
 * caller buffer of 3*n_verts doubles ordered on hip_stream (NULL = scene stream). */
ppn_status ppn_get_positions(ppn_scene* s, double* out_xyz);
ppn_status ppn_get_positions_dev(ppn_scene* s, void* out_dev, void* hip_stream);

/* Checkpoint / restore of the time-stepping state (positions, velocities),
 * [n_verts][3] each; set_state refuses non-finite values with PPN_ERR_STATE.
 * delta and the PDN countdown are per-step (Algorithm 1 resets them) and need
 * no saving. */
ppn_status ppn_get_state(ppn_scene* s, double* x, double* v);
ppn_status ppn_set_state(ppn_scene* s, const double* x, const double* v);

ppn_status ppn_get_last_stats(ppn_scene* s, ppn_step_stats* out);

/* Sizes of the loaded scene (any pointer may be NULL). */
ppn_status ppn_scene_info(ppn_scene* s, int32_t* n_verts, int32_t* n_tets, int32_t* n_edges,
                          int64_t* n_blocks, int64_t* device_bytes);

/* Message of the last failing call on this handle (or a global message when
 * s is NULL); valid until the next call on the handle. */
const char* ppn_last_error(const ppn_scene* s);

/* Kernel timing: when enabled, every 16th PCG matrix-product launch that does work
 * is bracketed by HIP events on the scene stream and summed into ms_spmv / n_spmv. */
ppn_status ppn_set_profiling(ppn_scene* s, int32_t enable);

/* ---- tracing ------------------------------------------------------------ */
/* Record one ppn_iter_record per Newton iteration of subsequent steps, plus
 * the projected element ids of each iteration. */
ppn_status ppn_set_trace(ppn_scene* s, int32_t enable);
/* Number of records of the last step. */
ppn_status ppn_trace_count(ppn_scene* s, int32_t* count);
/* Record i of the last step; proj_ids (nullable) receives rec->n_projected
 * ascending element ids. */
ppn_status ppn_trace_get(ppn_scene* s, int32_t i, ppn_iter_record* rec, int32_t* proj_ids);

/* ---- single stages on caller-given inputs (parity tests, benchmarks) ----- */
/* The state (x^n, v^n), targets and material of the scene define xhat and the
 * penalty terms; x is the iterate at which the stage is evaluated. */

/* Unprojected assembled gradient g [3 n_verts] at x (Sec. 3). */
ppn_status ppn_eval_gradient(ppn_scene* s, const double* x, double* g_out);

/* Element Hessians at x as full 12x12 row-major matrices for the element ids
 * ids[0..n) (nullable ids = all elements, n = n_tets); the projected ones
 * (proj_mask[e] != 0, nullable) after eigenvalue clamping (Sec. 3, Eq. (4)). */
ppn_status ppn_eval_element_hessians(ppn_scene* s, const double* x, const uint8_t* proj_mask,
                                     int32_t n, const int32_t* ids, double* H_out);

/* For callers that cannot allocate device memory during a call (code in tight
 * serving loops, harnesses that forbid hipMalloc): ppn_eval_element_hessians
 * with the same arguments, results and errors, except that its device staging
 * (the element ids and the 12x12 matrices before their copy to H_out) sits in
 * a fixed array of 4,734,976 bytes that the library holds once per GPU and process
 * instead of two allocations per call; the call allocates no device memory.
 * At most PPN_NOALLOC_MAX_ELEMENTS matrices per call (n, or n_tets when ids is
 * NULL); more return PPN_ERR_ARG with nothing evaluated.  Calls on one GPU
 * share the array and are serialised by the library (overlapping calls would
 * race on it); it keeps the last call's contents. */
#define PPN_NOALLOC_MAX_ELEMENTS 4096
ppn_status ppn_eval_element_hessians_noalloc(ppn_scene* s, const double* x, const uint8_t* proj_mask,
                                             int32_t n, const int32_t* ids, double* H_out);

/* Assembled global Hessian at x in 3x3 block-sparse row form, with the
 * elements in proj_mask (nullable) projected: row_ptr [n_verts+1],
 * col [n_blocks], vals [n_blocks][9] row-major blocks (Sec. 3, Sec. 4.1). */
ppn_status ppn_eval_hessian(ppn_scene* s, const double* x, const uint8_t* proj_mask,
                            int32_t* row_ptr, int32_t* col, double* vals);

/* Selection of Algorithm 1 (Sec. 4) on a caller-given assembled gradient g [3 n_verts]:
 * mask_out[e] = 1 iff proj_in[e] == 0 and (|S^e g|_inf > delta or
 * delta <= eps_delta).  count_out receives the number of ones. */
ppn_status ppn_select(ppn_scene* s, const double* g, double delta, const uint8_t* proj_in,
                      uint8_t* mask_out, int32_t* count_out);

/* One block-Jacobi PCG solve H dx = -g at x with proj_mask projected
 * (Sec. 4.1): returns dx [3 n_verts], the indefiniteness flag and the number
 * of products H d. */
ppn_status ppn_solve(ppn_scene* s, const double* x, const uint8_t* proj_mask, double* dx_out,
                     int32_t* ind_out, int32_t* iters_out);

/* The projections and solves of one Newton iteration from the iterate x
 * (Algorithm 1; for replaying a run iteration by iteration): the element
 * Hessians are evaluated at x, then PN projects every element, PDN (with its
 * countdown at 0) projects every element if the first solve reports
 * indefiniteness and solves again, and PPN runs the inner loop from
 * delta_in (INFINITY: not set yet, so the first round uses alpha |g|_inf).
 * mask_out [n_tets] receives the elements projected by the end of the
 * iteration, delta_out the delta carried to the next iteration (relaxed by
 * beta; delta_in for PN and PDN) and ind_out the final solve's
 * indefiniteness; any of them may be NULL.  x [3 n_verts]; the predictor
 * comes from the scene state, which the call leaves unchanged, as it leaves
 * the last step's statistics.  PPN_ERR_ARG for an unknown mode, a NULL x or
 * delta_in not > 0; PPN_ERR_STATE for a non-finite gradient at x. */
ppn_status ppn_debug_iterate(ppn_scene* s, int32_t mode, const double* x, double delta_in,
                             uint8_t* mask_out, double* delta_out, int32_t* ind_out);

/* Product q = H d [3 n_verts] with the assembled Hessian at x (Sec. 3; the
 * elements of proj_mask projected as in Eq. (5)). */
ppn_status ppn_hessian_product(ppn_scene* s, const double* x, const uint8_t* proj_mask,
                               const double* d, double* q_out);

/* Psi(x + gamma_k dx) - Psi(x) for n_gamma step sizes (the backtracking line
 * search of Sec. 5.1), evaluated term by term in FP64; out [n_gamma]. */
ppn_status ppn_energy_difference(ppn_scene* s, const double* x, const double* dx, int32_t n_gamma,
                                 const double* gammas, double* out);

/* Stateless batched projection (Sec. 3, Eq. (4)) of n symmetric 12x12 row-major
 * matrices in device memory: Hhat = H + sum_{lambda_i < eps} (eps - lambda_i) q_i q_i^T.
 * Precondition: every matrix is a linear-tetrahedron element Hessian, i.e.
 * symmetric and annihilating the three rigid translations (b_0 + b_1 + b_2 +
 * b_3 = 0, so in each row the four vertex columns of a coordinate sum to zero);
 * the solver deflates those exactly and clamps their zero eigenvalues to eps.
 * Both are checked first, to 1e-9 of each matrix's largest entry: a violation
 * (or a NaN) returns PPN_ERR_ARG with nothing written.  In and out may alias.
 * Runs on hip_stream (NULL = default stream) and returns after the kernels
 * finished; concurrent calls are serialised. */
ppn_status ppn_project_batch_dev(const double* H_dev, double* Hhat_dev, int64_t n, double eps,
                                 void* hip_stream);

/* A numbering of a mesh with spatial locality, to apply before
 * ppn_load_mesh (host-only; touches no device).  Writes vertex_order[n_verts]
 * and tet_order[n_tets], the input ids in their new order (new -> old), for
 * rest positions rest_xyz [n_verts][3] and tets [n_tets][4].  Vertex orders:
 *  PPN_ORDER_PENCIL: a banded sweep.  The axes are ranked by the mesh's
 *    extent, longest first; coordinates along the first two are rounded to
 *    the mesh spacing (the 10th percentile of the element edge lengths over
 *    a fixed-stride sample of at most 2^20 elements) and vertices sorted by
 *    them, then by the exact coordinate along the shortest axis.  On a
 *    regular grid this is the lexicographic numbering with the shortest axis
 *    fastest.
 *  PPN_ORDER_MORTON: the Z-order curve of the rest positions (21 bits per
 *    axis over the bounding box); adapts to graded meshes, with longer jumps.
 * Elements are sorted by their four new vertex ids (ascending, compared
 * lexicographically).  Ties keep the input order.  The caller renumbers its
 * arrays: new vertex v is old vertex_order[v], new element e is old element
 * tet_order[e] with each vertex id mapped old -> new.  The method's results
 * do not depend on the numbering up to rounding; the gathers of the PCG
 * product and of the element kernels do, and on a randomly numbered mesh the
 * product runs at a fraction of the rate a banded numbering gives.
 * PPN_ERR_ARG for a NULL pointer; PPN_ERR_MESH for an empty mesh, an unknown
 * kind, a non-finite position or a vertex index out of range. */
typedef enum { PPN_ORDER_PENCIL = 0, PPN_ORDER_MORTON = 1 } ppn_order_kind;
ppn_status ppn_locality_order(int32_t n_verts, const double* rest_xyz, int32_t n_tets,
                              const int32_t* tets, int32_t kind, int32_t* vertex_order,
                              int32_t* tet_order);


/* ---- Serving engine ---------------------------------------------------------
 * Many resident scenes stepped on request (time-step requests of uneven mesh
 * sizes as they arrive).  n_workers host threads take requests in arrival
 * order, skipping requests whose scene is busy; each resident scene has its
 * own HIP stream, so requests of different scenes run concurrently and their
 * kernels overlap on the device, while the requests of one scene run one at a
 * time in submission order.  A scene is admitted to device memory when its
 * footprint (exactly the bytes its buffers take) fits the budget; idle
 * resident scenes are evicted least recently used first, their positions and
 * velocities kept on the host until the scene is admitted again.  A scene's
 * arithmetic does not depend on what else runs: every result is bit-identical
 * to running the same requests alone.  The engine copies every input. */
typedef struct ppn_engine ppn_engine; /* opaque */

typedef struct {
  int32_t n_verts, n_tets;
  const double* rest_xyz;       /* [n_verts][3] */
  const int32_t* tets;          /* [n_tets][4], positively oriented at rest */
  const double* init_xyz;       /* [n_verts][3] or NULL (rest shape) */
  const double* init_vel;       /* [n_verts][3] or NULL (zero) */
  double rho;                   /* density [kg/m^3] */
  const double* E;              /* Young's modulus [Pa]: [n_tets] if per_element, else [1] */
  const double* nu;             /* Poisson ratio, same length as E */
  int32_t per_element;
  int32_t n_dirichlet;
  const int32_t* dirichlet_ids; /* [n_dirichlet] distinct vertex ids */
  double dt;                    /* time step [s] */
  double gravity[3];            /* [m/s^2] */
  int32_t precision;            /* ppn_precision */
  int32_t reserved0;
  const ppn_params* params;     /* NULL: ppn_params_default */
} ppn_scene_desc;

typedef struct {
  int64_t budget_bytes;    /* device-memory budget for resident scenes */
  int64_t resident_bytes;  /* footprint of the resident scenes */
  int64_t admissions;      /* scene loads into device memory */
  int64_t evictions;       /* scenes moved out to make room */
  int32_t resident_scenes, n_scenes, n_workers, pending;
  int64_t pcg_batches;         /* shared-launch PCG chunks run (batching on) */
  int64_t pcg_batched_solves;  /* solves carried by them */
  int64_t eval_launches;       /* shared evaluation / line-search phases run (PPN_BATCH_EVAL) */
  int64_t eval_batched_phases; /* scene phases carried by them */
} ppn_engine_info;

/* Create an engine on the current HIP device.  mem_budget_bytes <= 0 means 90%
 * of the device memory free at creation.  PPN_ERR_ARG unless 1 <= n_workers <= 256. */
ppn_status ppn_engine_create(ppn_engine** out, int32_t n_workers, int64_t mem_budget_bytes);
/* Waits for the running requests, drops the pending ones, frees everything. */
ppn_status ppn_engine_destroy(ppn_engine* e);
/* Register a scene (nothing is allocated on the device until its first
 * request); validates the description and builds its block pattern on the host.
 * PPN_ERR_MESH for an invalid mesh. */
ppn_status ppn_engine_add_scene(ppn_engine* e, const ppn_scene_desc* d, int32_t* scene_id_out);
/* Device bytes the scene takes while resident. */
ppn_status ppn_engine_scene_footprint(ppn_engine* e, int32_t scene_id, int64_t* bytes_out);
/* Queue one time step of scene_id in the given mode with the Dirichlet targets
 * of that step ([n_dirichlet][3], copied).  Returns at once. */
ppn_status ppn_engine_submit(ppn_engine* e, int32_t scene_id, int32_t mode, const double* targets,
                             int64_t* request_id_out);
/* Block until the request is done.  step_status_out receives the step's own
 * status (PPN_OK, a warning, or the error that ended it, with the message in
 * ppn_last_error(NULL) of the calling thread); stats_out its statistics;
 * latency_ms_out the time from submission to completion and queue_ms_out the
 * time it waited before a worker took it.  Any output may be NULL.  The
 * request's record is freed when its wait returns: a later wait on the same id
 * returns PPN_ERR_ARG (ids are never reused). */
ppn_status ppn_engine_wait(ppn_engine* e, int64_t request_id, ppn_status* step_status_out,
                           ppn_step_stats* stats_out, double* latency_ms_out, double* queue_ms_out);
/* Positions and velocities [n_verts][3] of a scene once all its submitted
 * requests are done (waits for them). */
ppn_status ppn_engine_get_state(ppn_engine* e, int32_t scene_id, double* x_out, double* v_out);
ppn_status ppn_engine_get_info(ppn_engine* e, ppn_engine_info* out);
/* Batched PCG (enable = 1): the solves of scenes being stepped at the same
 * time run in shared launches (one matrix-product and one update launch per
 * iteration for all of them, each workgroup working for one scene), which
 * removes the per-scene launch latency of small scenes.  Solves join and
 * leave the running batch at chunk boundaries (every 6 iterations).
 * Results are unchanged bit for bit.  Off by default.  PPN_ERR_STATE unless
 * the engine is idle. */
ppn_status ppn_engine_set_pcg_batching(ppn_engine* e, int32_t enable);
/* Shared launches across the scenes stepped at the same time (the per-element
 * parallelism of Sec. 4.1 carried across scenes): PPN_BATCH_PCG batches the
 * PCG solves as ppn_engine_set_pcg_batching(e, 1) does; adding PPN_BATCH_EVAL
 * also hands each Newton iteration's evaluation (element energies, gradients
 * and Hessians, assembly, gradient norms) and each line-search launch to one
 * thread that runs the phases of every scene waiting at that moment as one
 * launch per kernel over a table of the scenes.  Results are unchanged bit for
 * bit (every scene runs the same kernels with the same scene-local indices).
 * flags: 0, PPN_BATCH_PCG or PPN_BATCH_PCG | PPN_BATCH_EVAL (PPN_ERR_ARG
 * otherwise); PPN_ERR_STATE unless the engine is idle. */
#define PPN_BATCH_PCG 1
#define PPN_BATCH_EVAL 2
ppn_status ppn_engine_set_batching(ppn_engine* e, int32_t flags);

#ifdef __cplusplus
}
#endif

#endif /* PPN_H */
