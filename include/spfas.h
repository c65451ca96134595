/*
 * spfas -- nonlinear spectral multigrid (FAS) for heterogeneous nonlinear
 * diffusion, MI355X (gfx950) library.  C ABI.
 *
 * Method: Lee, Hamon, Castelletto, Vassilevski, White, "Nonlinear multigrid
 * based on local spectral coarsening for heterogeneous diffusion problems"
 * (arXiv 2005.01275).
 *
 * Problem (Section 2, eqs. model and kappa): find p with
 *     div q = f,   q = -K0(x) kappa(p) grad p   in Omega,
 *     p = g_D on the Dirichlet boundary,  -q.n = g_N on the Neumann boundary,
 * with kappa(p) = exp(alpha p), discretised by cell-centred two-point flux
 * finite volumes in mixed form (Section 2.1, eq. FV_matrix): one pressure per
 * cell, one flux per interior or Dirichlet face.
 *
 * Conventions for every entry point:
 *   - Return value: SPFAS_OK (0), SPFAS_NOT_CONVERGED (1, outputs written,
 *     see stats) or a negative error code.  On a negative code the outputs
 *     are left untouched and spfas_last_error() describes the failure.
 *   - No exceptions cross the ABI.  One handle must not be used by two
 *     threads at the same time.  Different handles are independent.
 *   - "stream" is a hipStream_t passed as void*; NULL means the default
 *     stream.  All device work of a call is enqueued on it; the calls below
 *     return after that work has completed (convergence is decided on the
 *     host), unless stated otherwise.
 *   - Arrays flagged SPFAS_MEM_DEVICE are device pointers on the current
 *     device; SPFAS_MEM_HOST arrays are ordinary host memory.  The caller
 *     keeps ownership of every array it passes.
 *   - Cell and face numbering of inputs and outputs is always the caller's
 *     ("input order").  Internal renumbering is invisible except through the
 *     parity hooks at the end of this header.
 */
#ifndef SPFAS_H
#define SPFAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPFAS_API_VERSION 1

typedef struct spfas_hierarchy spfas_hierarchy;   /* opaque; owns its device memory */

typedef enum {
  SPFAS_OK = 0,
  SPFAS_NOT_CONVERGED = 1,   /* max_it reached: state and stats written   */
  SPFAS_ERR_INVALID = -1,    /* bad argument or mesh; nothing written     */
  SPFAS_ERR_OOM = -2,        /* device allocation failed                  */
  SPFAS_ERR_DEVICE = -3,     /* HIP runtime error                         */
  SPFAS_ERR_NUMERIC = -4     /* non-finite residual, kappa or solve       */
} spfas_status;

typedef enum { SPFAS_MEM_HOST = 0, SPFAS_MEM_DEVICE = 1 } spfas_mem;
typedef enum { SPFAS_FACE_INTERIOR = 0, SPFAS_FACE_DIRICHLET = 1, SPFAS_FACE_NEUMANN = 2 } spfas_face_kind;
typedef enum { SPFAS_NEWTON = 0, SPFAS_PICARD = 1 } spfas_smoother;
typedef enum { SPFAS_PREC_FP64 = 0, SPFAS_PREC_MIXED = 1 } spfas_precision;

/*
 * Mesh (Section 2.1).  HOST memory, read during spfas_setup_hierarchy only.
 *   cell_volume   [n_cells]           |tau_K| > 0
 *   cell_centroid [n_cells*dim]       x_K, cell-major; also used to recover
 *                                     the lattice of a Cartesian mesh for box
 *                                     aggregation (distinct coordinate values
 *                                     per axis, exact comparison)
 *   cell_k0       [n_cells*dim*dim]   K0 of each cell, row-major
 *   face_cells    [2*n_faces]         (K, L) per face; L = -1 on the boundary.
 *                                     Interior faces are oriented K -> L and
 *                                     sigma > 0 means flow from K to L.
 *   face_area     [n_faces]           |eps|
 *   face_normal   [n_faces*dim]       unit normal pointing out of K
 *   face_point    [n_faces*dim]       collocation point x_eps
 *   face_kind     [n_faces]           spfas_face_kind
 * The half-transmissibilities of eq. half-transmissibility are computed from
 * these on the device and must be positive.
 */
typedef struct {
  int32_t dim;
  int64_t n_cells;
  int64_t n_faces;
  const double* cell_volume;
  const double* cell_centroid;
  const double* cell_k0;
  const int32_t* face_cells;
  const double* face_area;
  const double* face_normal;
  const double* face_point;
  const int8_t* face_kind;
} spfas_mesh;

/*
 * Device memory of a hierarchy.  When given, every device buffer the
 * hierarchy allocates (at setup and in later calls on the handle) comes from
 * alloc(bytes, stream, ctx) and is returned with free(ptr, bytes, stream,
 * ctx), where stream is the stream of the call that allocates; alloc returns
 * NULL on failure (the call then fails with ERR_OOM).  The callbacks may be
 * called from the thread that calls the library only, and must stay valid
 * until spfas_destroy returns.  Lets a framework's caching allocator (e.g.
 * PyTorch's) own the memory.  NULL allocator: hipMalloc / hipFree.
 */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, size_t bytes, void* stream, void* ctx);
  void* ctx;
} spfas_allocator;

/* How the cells of each level are grouped into aggregates (Section 3.1:
 * connected, non-overlapping aggregates; the paper partitions with METIS). */
typedef enum {
  SPFAS_AGG_BOX = 0,     /* boxes of box[] cells on the level lattice (Cartesian meshes) */
  SPFAS_AGG_USER = 1,    /* given by the caller for every coarsened level  */
  SPFAS_AGG_GREEDY = 2   /* greedy graph growth of about greedy_size cells   */
} spfas_agg_kind;

/*
 * Coarsening options (Section 3.1, Appendix A).
 *   n_levels  number of levels including the fine one (>= 1)
 *   box       BOX: aggregate edge per axis on each level's lattice; a
 *             remainder block with fewer than box/2 cells merges into its
 *             neighbour
 *   m         local eigenvectors kept per aggregate (m_A, uniform; clamped
 *             to the number of pressure unknowns of the aggregate)
 *   host_only nonzero: build only the host-side integer structure
 *             (aggregates and renumbering) without touching the GPU; only
 *             spfas_get_aggregation / spfas_get_permutation /
 *             spfas_level_sizes / spfas_destroy accept such a handle.
 *   agg_kind  spfas_agg_kind
 *   user_agg  USER: host array of the aggregate id of every cell of levels
 *             0 .. n_levels-2, concatenated (level l has as many cells as
 *             level l-1 has aggregates; level 0 is the mesh); ids of a level
 *             run over 0 .. n_agg-1, each used, each aggregate connected
 *             through the level's interior faces (ERR_INVALID otherwise)
 *   user_agg_len  number of entries of user_agg
 *   greedy_size   GREEDY: target aggregate size in cells of each level: seeds
 *             taken in ascending cell id grow breadth-first through
 *             neighbours in ascending id up to greedy_size cells; then every
 *             aggregate below greedy_size/2 cells, in ascending id, joins the
 *             neighbouring aggregate it shares the most interior faces with
 *             (ties: lower id); ids are compacted in ascending order
 *   greedy_size_coarse  GREEDY: the target on levels 1 and up (0: greedy_size);
 *             coarse cells carry several unknowns each, so a smaller target
 *             keeps the local problems of deeper levels small
 *   eig_threshold  > 0: the number of eigenvectors of each aggregate is
 *             the number of eigenvalues of its local problem (eq.
 *             local-eigenvalue-problem, lambda_1 = 0 included) up to
 *             eig_threshold times its largest eigenvalue, clamped to
 *             [m_min, m] and to the aggregate's unknowns; a varying count
 *             per aggregate is allowed by Appendix A (m_A per aggregate).
 *             The setup then solves each level's eigenproblems once more to
 *             count before it builds the coarser level.  Not with
 *             host_only.  <= 0: the uniform m above.
 *   m_min     lower clamp of the threshold count (1 <= m_min <= m)
 *   m_f       coarse flux unknowns per coarse interface (Appendix A, the
 *             edge-based flux space): 1, the PV trace only (0 means 1).
 *             Several traces per interface (eigenvector traces on extended
 *             aggregates with an SVD) are not built: other values are
 *             rejected with ERR_INVALID.
 */
typedef struct {
  int32_t n_levels;
  int32_t box[3];
  int32_t m;
  int32_t host_only;
  int32_t agg_kind;
  const int32_t* user_agg;
  int64_t user_agg_len;
  int32_t greedy_size;
  double eig_threshold;
  int32_t m_min;
  int32_t m_f;
  int32_t greedy_size_coarse;
} spfas_coarsen_opts;

/*
 * Problem data of one solve (Section 2, eq. model).
 *   alpha        kappa(p) = exp(alpha p)
 *   source       [n_cells]  density f (multiplied by |tau_K| internally)
 *   g_dirichlet  [n_faces]  g_D, read on Dirichlet faces; NULL means 0
 *   g_neumann    [n_faces]  g_N = -q.n, read on Neumann faces; NULL means 0
 *   mem          where the arrays live (source, g_*, shift)
 * kappa family (a zero-initialised tail gives the exponential above):
 *   kappa_kind   SPFAS_KAPPA_EXP: kappa(psi) = exp(alpha psi);
 *                SPFAS_KAPPA_RICHARDS: kappa(psi) = a / (a + |psi|^beta)
 *                (Example 3, eq. permeability_function_richards), with
 *                kappa_a > 0 and kappa_beta >= 1
 *   shift        [n_cells] or NULL: kappa is evaluated at psi = p - shift
 *                (Example 3: p = psi + z, shift = the height z).  Coarse
 *                levels use the volume-weighted mean of the shift over the
 *                level-0 cells of each coarse cell, at the aggregate-mean
 *                pressure of Prop. 1.
 * The cap of spfas_solve_opts.dp_cap is the caller's: ln(c)/alpha belongs
 * to the exponential family (Section 4.1); pass 0 (no cap) for the other.
 */
typedef enum { SPFAS_KAPPA_EXP = 0, SPFAS_KAPPA_RICHARDS = 1 } spfas_kappa_kind;

typedef struct {
  double alpha;
  const double* source;
  const double* g_dirichlet;
  const double* g_neumann;
  int32_t mem;
  int32_t kappa_kind;
  double kappa_a;
  double kappa_beta;
  const double* shift;
} spfas_problem;

/*
 * Solve options (Section 4 and Alg. 1).
 *   smoother            SPFAS_NEWTON or SPFAS_PICARD (FAS only; the
 *                       single-level entry points fix it by name)
 *   rtol, atol          stop when ||r(x)||_2 <= max(rtol*||r(x0)||_2, atol)
 *   max_it              V-cycles (FAS) or nonlinear steps (single level)
 *   bt_nmax, bt_theta   Alg. 1 parameters (paper: 4 and 0.9)
 *   dp_cap              max |delta p| per smoothing step, ln(c)/alpha in the
 *                       paper (c = 1.5 or 5); <= 0 disables the cap
 *   coarsest_max_steps  smoothing steps on the coarsest level (paper: 10)
 *   lin_rtol, lin_max_it  inner Krylov tolerance and iteration limit of
 *                       one linear solve (PCG and its BiCGStab fallback
 *                       together)
 *   x0_given            nonzero: p and sigma hold the initial guess on entry
 *   lin_rtol_coarse     inner tolerance on coarse levels (<= 0: lin_rtol)
 *   lin_target          > 0: a level-0 smoothing step at residual norm r
 *                       solves to max(lin_rtol, min(0.1, lin_target*tol/r)),
 *                       tol being the outer stopping threshold, so the last
 *                       steps are not solved far below what the stop needs
 *                       (inexact Newton forcing; the paper leaves the inner
 *                       tolerance open); 0 = off
 *   newton_pcg          nonzero: Newton systems are first tried with PCG
 *                       (they are nearly symmetric: the non-symmetric part
 *                       is the kappa' term of E), falling back to BiCGStab
 *                       from scratch on a breakdown, on a stall (||r||
 *                       lowered less than 2x over 5 iterations) or
 *                       without convergence, with the iterations the limit
 *                       has left; 0: BiCGStab only
 *   amg_reuse           > 0: the AMG values of a level's preconditioner are
 *                       kept for up to amg_reuse further linearisations of
 *                       the same solve (< 0: no limit), as long as its
 *                       Krylov solves take at most f + max(2, f/2)
 *                       iterations, f being the count right after the values
 *                       were last recomputed; the Krylov products always use
 *                       the current matrix, so only the inner iteration
 *                       changes, never the system solved.  0: recomputed
 *                       after every linearisation
 *   lin_max_it_coarse   iteration limit of each coarse-level linear solve
 *                       (<= 0: lin_max_it); a solve that reaches it hands
 *                       its current iterate to the smoothing step, whose
 *                       direction Alg. 1 then checks
 *   coarsest_atol       absolute tolerance of the coarsest level's own
 *                       convergence test (Section 4: relative 1e-8 or
 *                       absolute 1e-10); < 0: atol.  Lets the outer solve run
 *                       with atol = 0 (a pure relative stop) while the
 *                       coarsest level keeps the paper's absolute floor
 *   precision           SPFAS_PREC_FP64, or SPFAS_PREC_MIXED: the level-0
 *                       linearised systems are stored (S in its SELL layout
 *                       and the right-hand side) and solved (Krylov vectors,
 *                       AMG cycle input and output) in FP32, while the
 *                       residual, the Jacobian entries, the flux
 *                       back-substitution, Alg. 1 and the state update stay
 *                       FP64: every smoothing step corrects the FP64 defect,
 *                       so the solve reaches the same FP64 root.  Coarse
 *                       levels are unchanged (FP64).  A level-0 AMG that is
 *                       not classical keeps the FP64 path.
 */
typedef struct {
  int32_t smoother;
  double rtol;
  double atol;
  int32_t max_it;
  int32_t bt_nmax;
  double bt_theta;
  double dp_cap;
  int32_t coarsest_max_steps;
  double lin_rtol;
  int32_t lin_max_it;
  int32_t x0_given;
  double lin_rtol_coarse;
  double lin_target;
  int32_t newton_pcg;
  int32_t amg_reuse;
  int32_t lin_max_it_coarse;
  double coarsest_atol;
  int32_t precision;
} spfas_solve_opts;

typedef struct {
  int32_t iterations;       /* V-cycles or nonlinear steps taken            */
  int32_t lin_iters;        /* Krylov iterations summed over all solves     */
  int32_t bt_halvings;      /* step halvings taken by Alg. 1                */
  int32_t smoothing_steps;  /* smoothing steps on all levels                */
  int32_t stopped_after_presmooth;  /* last V-cycle ended after pre-smoothing */
  double r0;                /* ||r(x0)||                                    */
  double r_final;           /* ||r(x)|| on return                          */
  double solve_ms;          /* wall time of the call (host clock)           */
  int32_t rejected_steps;   /* smoothing steps dropped because the linearised
                               system or its solve was not finite            */
  int32_t refine_steps;     /* mixed precision: FP32 correction solves of the
                               level-0 iterative refinement                  */
} spfas_stats;

/* Fills *o with the paper's settings (Section 4): Newton, rtol 1e-8, atol
 * 1e-10, max_it 50, n_max 4, theta 0.9, no cap, 10 coarsest steps (coarsest
 * atol = atol), inner rtol 1e-8 and 500 inner iterations, x0 = 0. */
void spfas_default_solve_opts(spfas_solve_opts* o);

/*
 * Builds the multilevel hierarchy (Section 3.1, Appendix A; Prop. 1 for the
 * static coarse local matrices; Appendix B for the projector weights):
 * half-transmissibilities, aggregation and renumbering on the host, then
 * batched on the device the local spectral problems, PV traces, trace
 * extensions, bubbles, P_sigma, P_p, Q and M^{l+1}_A, D^{l+1}_A.  The
 * hierarchy depends on the mesh only and serves any number of solves.
 * allocator: see spfas_allocator; NULL for hipMalloc / hipFree.
 * Errors: ERR_INVALID for a malformed mesh (index out of range, non-positive
 * volume, face area or half-transmissibility, a non-finite centroid, no
 * Dirichlet face, n_levels < 1, a lattice
 * that cannot be recovered from the centroids for BOX, a malformed USER
 * aggregation), ERR_OOM, ERR_DEVICE.
 * *out receives a handle to be released with spfas_destroy.
 */
int spfas_setup_hierarchy(const spfas_mesh* mesh, const spfas_coarsen_opts* opts,
                          const spfas_allocator* allocator, void* stream, spfas_hierarchy** out);

/* Device bytes the hierarchy holds now (*bytes) and at most held so far
 * (*peak), counting everything allocated through its allocator. */
int spfas_hierarchy_device_bytes(const spfas_hierarchy* h, int64_t* bytes, int64_t* peak);

/* Sets the peak that spfas_hierarchy_device_bytes reports to the bytes held
 * now, so that the peak of what follows (a solve's temporaries) can be
 * measured.  Not to be called while a solve on h is running. */
int spfas_hierarchy_reset_peak(spfas_hierarchy* h);

/*
 * Solves the nonlinear system (eq. nonlinear_system_residual_form) with FAS
 * V-cycles (Alg. 2): Picard or Newton smoothing with the step cap and Alg. 1,
 * restriction R = P^T, projection Q, coarse problems
 * r^{l+1}(y) = A^{l+1}(y) - [A^{l+1}(Q x) - R r^l(x)] (eq.
 * coarse_level_residual) built from the coarse local matrices without
 * visiting the fine level, and at most coarsest_max_steps smoothing steps on
 * the coarsest level (fewer when its residual falls to rtol times its value
 * on entry, or to atol, or after a step Alg. 1 rejected).
 *   p      [n_cells]  in: initial guess if x0_given; out: pressure
 *   sigma  [n_faces]  in: initial guess if x0_given (Neumann entries
 *                     ignored); out: flux of every face, -|eps| g_N on
 *                     Neumann faces
 *   state_mem  where p and sigma live
 *   stats      may be NULL
 * Returns OK, NOT_CONVERGED (state written), ERR_INVALID, ERR_NUMERIC
 * (state untouched), ERR_DEVICE.
 */
int spfas_fas_solve(spfas_hierarchy* h, const spfas_problem* prob, const spfas_solve_opts* opts,
                    double* p, double* sigma, int32_t state_mem, spfas_stats* stats, void* stream);

/* Single-level Picard iteration (Section 2.2; Section 3.3 for the Picard
 * system) on the fine level with the same cap and Alg. 1.  Arguments and
 * errors as spfas_fas_solve; opts->smoother is ignored. */
int spfas_picard_solve(spfas_hierarchy* h, const spfas_problem* prob, const spfas_solve_opts* opts,
                       double* p, double* sigma, int32_t state_mem, spfas_stats* stats, void* stream);

/* Single-level Newton iteration (Section 2.2; Jacobian of Section 3.3,
 * Prop. 3 on the fine level).  As spfas_picard_solve. */
int spfas_newton_solve(spfas_hierarchy* h, const spfas_problem* prob, const spfas_solve_opts* opts,
                       double* p, double* sigma, int32_t state_mem, spfas_stats* stats, void* stream);

/* Nonlinear cascadic multigrid (Section 4.2, Table 4): the right-hand side
 * is restricted to every level (b^{l+1} = R b^l = P^T b^l), the coarsest
 * problem is solved from zero with smoothing steps (opts->smoother, the cap
 * and Alg. 1 as in spfas_fas_solve) until it converges, and each finer level
 * starts from the prolongated (P) solution of the level below and is
 * smoothed until it converges, up to level 0.  "Converges" on level l means
 * ||r^l|| <= max(rtol ||b^l||, atol), with at most max_it smoothing steps per
 * level; a level also stops after a step that Alg. 1 rejected (state
 * unchanged), and hands its state up either way.
 * p, sigma: as spfas_fas_solve, outputs only; opts->x0_given must be 0
 * (ERR_INVALID otherwise).  level_steps: host array of n_levels int32, the
 * smoothing steps taken on each level (finest first), or NULL.
 * stats->iterations counts the level-0 steps, stats->r0 = ||b^0||.
 * Returns SPFAS_OK when level 0 converged, SPFAS_NOT_CONVERGED when it
 * reached max_it; other errors as spfas_fas_solve. */
int spfas_cascadic_solve(spfas_hierarchy* h, const spfas_problem* prob, const spfas_solve_opts* opts,
                         double* p, double* sigma, int32_t state_mem, spfas_stats* stats, int32_t* level_steps,
                         void* stream);

/*
 * Fine-level residual r(x) = A(x) - b (eqs. fine_level_residual and
 * fine_level_operators) at the state (p, sigma), written in input order:
 *   r_p     [n_cells]  D sigma + f
 *   r_sigma [n_faces]  M(p) sigma + D^T p + g; 0 on Neumann faces
 * All four arrays live in `mem`.
 */
int spfas_eval_residual(spfas_hierarchy* h, const spfas_problem* prob, const double* p,
                        const double* sigma, double* r_p, double* r_sigma, int32_t mem, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * fine-level residual of spfas_eval_residual, on DEVICE arrays only
 * (prob->mem must be SPFAS_MEM_DEVICE; p, sigma, r_p, r_sigma are device
 * pointers in input order, as in spfas_eval_residual with mem =
 * SPFAS_MEM_DEVICE), computed with no hipMalloc, hipFree or other allocating
 * call.  The state and the residual in internal order are staged in a
 * static device array of 96 MiB that the library holds on each device it
 * runs on until the process ends; the level-0 problem may have at most
 * 6,291,456 unknowns (flux + cells), larger ones are rejected with
 * ERR_INVALID before any work, and so is a problem with a kappa shift
 * (prob->shift must be NULL).  The current device must be the one the
 * hierarchy was built on (ERR_INVALID otherwise).  All calls on one GPU
 * share that array: calls that overlap in time on one GPU (on any stream or
 * thread, any hierarchy) race and must not be made.  Returns after the work
 * has completed.
 */
int spfas_eval_residual_noalloc(spfas_hierarchy* h, const spfas_problem* prob, const double* p,
                                const double* sigma, double* r_p, double* r_sigma, void* stream);

/* ------------------------------------------------------------------ serving
 * Continuous batching of solve requests on one GPU.  Models (a mesh and its
 * coarsening options) are registered once; their hierarchies are built on
 * first use and kept in device memory.  A fixed number of worker threads,
 * each with its own HIP stream, take requests from one queue: a request is
 * admitted as soon as a worker is free and its model's hierarchy is cached
 * and idle, or can be built within the device-memory budget (idle
 * hierarchies of other models are evicted, least recently used first, to
 * make room; the footprint of a model is estimated from its sizes until its
 * first build measures it).  Requests that cannot be admitted yet do not
 * hold back later ones.  Solves of different requests overlap on the GPU; a
 * request's result does not depend on what else is in flight.  Each model
 * has at most one cached hierarchy: requests on the same model run one
 * after the other.  All problem data and results are host memory.  Server
 * functions are thread-safe; errors are reported by
 * spfas_server_last_error().
 */
typedef struct spfas_server spfas_server;

typedef struct {
  int32_t n_slots;       /* worker threads = solves in flight (1..64)                */
  int64_t hbm_budget;    /* device bytes for cached hierarchies; <= 0: 80% of free */
  int32_t device;        /* HIP device ordinal                                      */
} spfas_server_opts;

typedef enum { SPFAS_SOLVE_FAS = 0, SPFAS_SOLVE_NEWTON = 1, SPFAS_SOLVE_PICARD = 2 } spfas_solve_kind;

typedef struct {
  double queue_ms;       /* submission to admission                     */
  double setup_ms;       /* hierarchy build (0 on a cache hit)          */
  double solve_ms;       /* the solve, host state copies included       */
  double total_ms;       /* submission to completion                    */
  int32_t cache_hit;     /* the hierarchy was already cached            */
} spfas_request_info;

typedef struct {
  int64_t submitted, completed, setups, cache_hits, evictions;
  int64_t peak_bytes;    /* largest device bytes held by cached hierarchies */
  int64_t cached_bytes;  /* held now                                         */
  int64_t budget_bytes;
} spfas_server_counters;

int spfas_server_create(const spfas_server_opts* opts, spfas_server** out);

/* Registers a model; the mesh (and a USER aggregation) is copied. */
int spfas_server_add_model(spfas_server* s, const spfas_mesh* mesh, const spfas_coarsen_opts* coarsen,
                           int64_t* model_id);

/* Queues one solve (kind: spfas_solve_kind) of the model from x0 = 0; the
 * problem arrays (host) are copied.  Returns at once with a ticket. */
int spfas_server_submit(spfas_server* s, int64_t model_id, const spfas_problem* prob, const spfas_solve_opts* opts,
                        int32_t kind, int64_t* ticket);

/* Blocks until the ticket's solve is done, then writes p [n_cells] and
 * sigma [n_faces] (host, input order; either may be NULL), stats and info
 * (may be NULL) and releases the ticket.  Returns the solve's status
 * (ERR_OOM when the model cannot fit under the budget at all). */
int spfas_server_wait(spfas_server* s, int64_t ticket, double* p, double* sigma, spfas_stats* stats,
                      spfas_request_info* info);

int spfas_server_counters_get(spfas_server* s, spfas_server_counters* counters);

/* Stops the workers and releases every hierarchy; collect every ticket
 * first. */
void spfas_server_destroy(spfas_server* s);

const char* spfas_server_last_error(void);

/* ------------------------------------------------------------------ parity hooks
 * Read-only views of the hierarchy used to compare it with an independent
 * implementation.  "Canonical order" on level 0 is the input order of
 * cells and of the non-Neumann faces; on level l+1 it is the aggregate id
 * (boxes numbered lexicographically, x fastest) for cells and, for flux
 * unknowns: interfaces between aggregates A < B sorted by (A, B), then
 * Dirichlet groups by A, then bubbles by (A, j).  Pressure unknowns of a
 * cell are consecutive.  All outputs are HOST arrays.
 */

/* Sizes of level l: cells, pressure unknowns, flux unknowns. */
int spfas_level_sizes(const spfas_hierarchy* h, int32_t level, int64_t* n_cells, int64_t* n_p,
                      int64_t* n_flux);

/* agg[n_cells(level)]: canonical aggregate id of each canonical cell of
 * `level` (0 <= level < n_levels-1). */
int spfas_get_aggregation(const spfas_hierarchy* h, int32_t level, int32_t* agg);

/* Renumbering of `level` (0 <= level < n_levels-1): cell_order[n_cells] and
 * flux_order[n_flux] give, for each internal position, the canonical id.
 * Cells are contiguous per aggregate; flux unknowns are grouped inside-
 * aggregate / per interface / Dirichlet. */
int spfas_get_permutation(const spfas_hierarchy* h, int32_t level, int32_t* cell_order,
                          int32_t* flux_order);

typedef enum {
  SPFAS_OP_EIGVALS = 0,  /* level l: the m_A smallest eigenvalues of each aggregate's L_A, ascending, aggregates in canonical order */
  SPFAS_OP_PP = 1,       /* level l: P_A blocks (n_pA x m_A, row-major), canonical aggregate order          */
  SPFAS_OP_PSIGMA = 2,   /* level l: P_sigma as dense [n_flux(l) x n_flux(l+1)], row-major, canonical      */
  SPFAS_OP_MLOC = 3,     /* level l+1: static M^{l+1}_A blocks (k_A x k_A, row-major), canonical order     */
  SPFAS_OP_DLOC = 4,     /* level l+1: D^{l+1}_A blocks (m_A x k_A, row-major), canonical order            */
  SPFAS_OP_W = 5,        /* level l+1: projector weights w_A, concatenated, canonical order                */
  SPFAS_OP_QSIGMA = 6,   /* level l: Q_sigma as dense [n_flux(l+1) x n_flux(l)], row-major, canonical      */
  SPFAS_OP_MCOUNT = 7    /* level l: m_A of each aggregate (as doubles), canonical aggregate order         */
} spfas_level_op;

/* Copies the operator `what` between `level` and level+1 into out[count]
 * (count must equal the exact size, else ERR_INVALID reports the size
 * needed).  Dense P_sigma / Q_sigma are meant for small test problems. */
int spfas_get_level_operator(const spfas_hierarchy* h, int32_t level, int32_t what, double* out,
                             size_t count);

/* ------------------------------------------------------------------ measurement
 * Kernel timing with HIP events recorded on the stream of the solve calls.
 * Each instrumented launch is bracketed by two events; `algo_bytes` is the
 * algorithmic HBM traffic of the launches (the minimum the method moves:
 * per flux unknown F, cell N and cell-face incidence I of level 0,
 * residual 40F + 20N + 4I, at a trial point x + s dx 48F + 28N + 4I (also for
 * the multi-step pass, which reads the same data once), Newton
 * linearisation 40F + 36N + 12I; with E = stored nonzeros of S including the
 * diagonal: S x with its dot products 12E + 24N (FP64 value + int32
 * column per entry); on the finest level of the classical AMG (FP16 value
 * + int32 column per stored entry, N_c coarse points, E_w = E, E_R =
 * entries of P, E_AP = entries of A P; the cycle's input and output are
 * FP64, its residual and coarse vectors FP32): pre-sweep + residual
 * 6E_w + 12N, restriction 6E_R + 4N + 4N_c, prolongation + sweep
 * 6E_AP + 28N + 4N_c).
 */
typedef enum {
  SPFAS_PROF_FINE_RESID = 0,         /* fine residual, also inside Alg. 1 trials   */
  SPFAS_PROF_FINE_LINEARIZE = 1,     /* S = D M^{-1} E and its right-hand side      */
  SPFAS_PROF_FINE_SPMV = 2,          /* S x (+ one dot) in the fine-level Krylov solver */
  SPFAS_PROF_FINE_AMG_DOWN = 3,      /* finest AMG level: pre-smoothing + residual  */
  SPFAS_PROF_FINE_AMG_RESTRICT = 4,  /* finest AMG level: restriction               */
  SPFAS_PROF_FINE_AMG_UP = 5,        /* finest AMG level: prolongation + smoothing  */
  SPFAS_PROF_FINE_SPMV2 = 6,         /* S x (+ two dots), second product of BiCGStab */
  SPFAS_PROF_FINE_RESID_TRIALS = 7,  /* fine residual norms at up to 4 step lengths in one pass (Alg. 1 halvings) */
  SPFAS_PROF_AMG_TAIL_DOWN = 8,      /* the same three phases summed over the level-0 AMG's levels below the */
  SPFAS_PROF_AMG_TAIL_RESTRICT = 9,  /*   finest (FP32 vectors: pre-sweep 6E + 8N, restriction 6E_R + 4N +  */
  SPFAS_PROF_AMG_TAIL_UP = 10,       /*   4N_c, prolongation + sweep 6E_AP + 20N + 4N_c per level)          */
  SPFAS_PROF_COUNT = 11
} spfas_prof_kernel;

/* Turns the timing on (nonzero) or off and clears the counters. */
int spfas_profile_enable(spfas_hierarchy* h, int32_t enable);

/* Totals since the last enable: number of launches, summed event time in
 * milliseconds and summed algorithmic bytes.  Synchronises the stream. */
int spfas_profile_read(spfas_hierarchy* h, int32_t which, int64_t* launches, double* total_ms,
                       double* algo_bytes);

/* Releases every resource of the handle (NULL is allowed). */
void spfas_destroy(spfas_hierarchy* h);

/* Message of the last failed call on this thread; valid until the next
 * call on this thread.  Never NULL. */
const char* spfas_last_error(void);

int spfas_version(void);

#ifdef __cplusplus
}
#endif
#endif
