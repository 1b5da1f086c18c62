/*
 * vps.h -- C-ABI of the MI355X (gfx950) vertex-patch multigrid library.
 *
 * Method: arXiv 2405.19004, "An implementation of tensor product patch smoothers
 * on GPU".  Q_k finite elements for -Laplace(u) = f on the unit square (d = 2)
 * or cube (d = 3), u = 0 on the boundary (Sec. 2, eq:model, eq:weak_form,
 * eq:matrix-def); geometric multigrid V-cycle (Alg. 1) whose smoother is the
 * colourised multiplicative vertex-patch Schwarz method (Sec. 2.2, Alg. 3) with
 * local solves by fast diagonalisation (Sec. 2.4, eq:inverse2d/3d); matrix-free
 * sum-factorised operator (Sec. 2.3, eq:mf); prolongation by embedding and
 * restriction as its transpose (Sec. 2.1).
 *
 * Mesh and vectors
 *   Level l has 2^l cells per direction, h = 2^-l, n1d = k*2^l + 1 nodes per
 *   direction, N = n1d^d nodes (boundary nodes included).  Level 1 is the
 *   coarsest level: its single vertex patch covers every interior DoF, so one
 *   patch solve is the exact coarse solve (Sec. 2.1).
 *   A level vector is a dense device array of N values, lexicographic with x0
 *   fastest (index = i0 + n1d*(i1 + n1d*i2)), support points = Gauss-Lobatto.
 *   Boundary entries are ignored on input (treated as 0).  Functions that
 *   produce a fresh vector (operator, residual, restriction, rhs) write 0 to
 *   the boundary entries; in/out vectors (smoother x, prolongate-add x) keep
 *   their boundary entries untouched.
 *   `prec` selects the element type of every vector argument of the call:
 *   VPS_FP64 -> double, VPS_FP32 -> float.
 *
 * Ownership, streams, errors
 *   Vectors are caller-owned device pointers (for example torch tensors,
 *   contiguous).  The library owns the hierarchy, tables and scratch vectors it
 *   allocates in vps_create and frees in vps_destroy.  All device work is
 *   enqueued on the stream given to vps_create (0 = the null stream) and is
 *   asynchronous, except where a function says it synchronises.  Distinct
 *   problems may be used from distinct host threads; one problem must not be
 *   used by two host threads at once.  Every function returns VPS_OK (0) or a
 *   negative status; vps_last_error() returns the message of the last failure
 *   on the calling thread.  No call aborts the process.
 */
#ifndef VPS_H
#define VPS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum vps_status {
  VPS_OK = 0,
  VPS_EINVAL = -1,      /* invalid argument (dimension, degree, level, pointer, size) */
  VPS_ENOMEM = -2,      /* device or host allocation failed */
  VPS_EHIP = -3,        /* a HIP runtime call failed; message names it */
  VPS_ENOCONV = -4,     /* iteration limit reached before the tolerance */
  VPS_EBREAKDOWN = -5,  /* CG breakdown: p^T A p <= 0 or a non-finite scalar */
  VPS_ENOTFINITE = -6,  /* non-finite input (right-hand side) */
  VPS_EBUSY = -7        /* server: request can never fit the memory budget, or queue full */
};

enum vps_prec { VPS_FP64 = 0, VPS_FP32 = 1 };
enum vps_smooth {
  VPS_MULTIPLICATIVE = 0,
  VPS_ADDITIVE = 1,
  VPS_MULTIPLICATIVE_BOUNDARY = 2,
  VPS_MULTIPLICATIVE_SEPARATE = 3,
  VPS_MULTIPLICATIVE_MFMA = 4
};
enum vps_solve { VPS_SOLVE_FP64 = 0, VPS_SOLVE_MIXED = 1 };

/* vps_create flags */
#define VPS_FLAG_FP64_HIERARCHY 0x1u /* allocate FP64 V-cycle scratch (needed by FP64 vcycle / FP64 solve) */
#define VPS_FLAG_FP32_HIERARCHY 0x2u /* allocate FP32 V-cycle scratch (needed by FP32 vcycle / mixed solve) */
#define VPS_FLAG_NO_SOLVER 0x4u      /* skip the outer-CG vectors (vps_pcg_solve then fails with VPS_EINVAL) */
#define VPS_FLAG_POST_SAME_ORDER 0x8u /* post-smoothing colours ascending (Alg. 1 read literally; the
                                         V-cycle is then not symmetric and vps_pcg_solve uses the flexible
                                         beta in both modes).  Default: descending (symmetric V-cycle). */
#define VPS_FLAG_BOUNDARY_SMOOTHER 0x10u /* V-cycles smooth with the "Boundary" kernel
                                            (VPS_MULTIPLICATIVE_BOUNDARY below; Sec. 4.1.3) */
#define VPS_FLAG_SEPARATE_SMOOTHER 0x40u /* V-cycles smooth in the "Separate" form
                                            (VPS_MULTIPLICATIVE_SEPARATE below; Sec. 4.1, Table 6) */
#define VPS_FLAG_MFMA_SMOOTHER 0x80u /* V-cycles smooth with VPS_MULTIPLICATIVE_MFMA (below) */
#define VPS_FLAG_GRAPHS 0x20u /* replay the CG preconditioner from a HIP graph captured on first use
                                 instead of launching its kernels one by one (same results; measured
                                 slower than direct launches for these solves, so off by default) */

typedef struct vps_problem vps_problem;

typedef struct {
  int dim, degree, level;
  long long n1d, n_dofs, n_interior, n_cells, n_patches;
  int n_colors;
  long long color_count[8];
  double h;
} vps_level_info_t;

typedef struct {
  int iterations;                 /* CG iterations performed */
  double rel_residual;            /* recursively updated ||r||_2 / ||b||_2 at exit */
  double true_rel_residual;       /* ||b - A x||_2 / ||b||_2 recomputed in FP64 at exit */
  int status;                     /* VPS_OK, VPS_ENOCONV, VPS_EBREAKDOWN or VPS_ENOTFINITE */
} vps_solve_stats_t;

/* Create the level hierarchy 1..fine_level for Q_degree in `dim` dimensions.
 * dim in {2,3}, degree in 1..7, fine_level >= 1 and N(fine_level) < 2^40.
 * Builds the 1D tables on the host (Gauss-Lobatto nodes, Gauss quadrature,
 * reference stiffness/mass, the generalised eigenpairs of eq:fast_inverse),
 * uploads them, and allocates scratch per `flags`.  hip_stream is a
 * hipStream_t (may be NULL).  *out receives the handle. */
int vps_create(int dim, int degree, int fine_level, unsigned flags, void* hip_stream, vps_problem** out);

/* Free everything vps_create allocated (synchronises the problem's stream).  NULL is a no-op. */
int vps_destroy(vps_problem* p);

/* Device bytes vps_create would allocate for these arguments (host-only, no device call). */
int vps_footprint_bytes(int dim, int degree, int fine_level, unsigned flags, size_t* bytes);

/* Sizes and per-colour patch counts of `level` (1..fine_level).  Host-only. */
int vps_level_info(const vps_problem* p, int level, vps_level_info_t* out);

/* Flat index of node coords[0..dim-1] (coords[a] along axis a, 0..n1d-1) on `level`.  Host-only. */
int vps_dof_index(const vps_problem* p, int level, const int* coords, long long* idx);

/* First closure index of every patch of `color` on `level` (Sec. 3.1.2: one index per patch,
 * the rest follows from strides), written to host array out[0..cap-1] in launch order;
 * *n receives the patch count of the colour (also when cap is smaller).  Host-only. */
int vps_patch_first_index(const vps_problem* p, int level, int color, long long* out, long long cap, long long* n);

/* y = A_level x (eq:linear_system, matrix-free, Sec. 2.3 eq:mf). */
int vps_operator_apply(vps_problem* p, int level, int prec, const void* x, void* y);

/* r = b - A_level x (the residual step of Alg. 1). */
int vps_residual(vps_problem* p, int level, int prec, const void* b, const void* x, void* r);

/* One application of the vertex-patch smoother on `level`.
 * VPS_MULTIPLICATIVE: x <- S_level(x, b), Alg. 3: colours in ascending order
 *   (descending when reverse_colors != 0); for every patch j of the colour,
 *   x_j^I += A_j^{-1}(b_j^I - Abar_j x_j) with the localised residual of Sec. 2.2.
 * VPS_ADDITIVE: x += sum_j R_j^T A_j^{-1} R_j b (b is a residual; undamped; the
 *   colours only order the accumulation, the result does not depend on them
 *   beyond rounding).
 * VPS_MULTIPLICATIVE_BOUNDARY: the multiplicative smoother computed as in Sec. 4.1.3
 *   (eq:A_ib_2d/3d): since A_j^{-1} is exact, x_j^I <- A_j^{-1}(b_j^I - A^{IB} x_j^B); the old
 *   interior values are never read.  Equal to VPS_MULTIPLICATIVE up to rounding.
 * VPS_MULTIPLICATIVE_SEPARATE: the multiplicative smoother as two kernels per colour (the
 *   "Separate" kernels of Sec. 4.1, Table 6): the residual b - A x by the operator kernel into
 *   the level's residual buffer, then x^I += A_j^{-1} r^I.  Needs the hierarchy flag of `prec`.
 *   Equal to VPS_MULTIPLICATIVE up to rounding.
 * VPS_MULTIPLICATIVE_MFMA: VPS_MULTIPLICATIVE with the three contractions of the localised
 *   residual (Sec. 3.1.1) on the matrix cores, for 3D degree 4 in FP32 on launches of at least
 *   1024 workgroups; every other case runs VPS_MULTIPLICATIVE.  Equal to it up to rounding
 *   (a measured variant: slower than the vector form here). */
int vps_smoother_apply(vps_problem* p, int level, int prec, int mode, int reverse_colors, const void* b, void* x);

/* One colour of Alg. 3 (mode as above) on `level`; color in 0..2^dim-1 where the colour of the
 * patch at interior vertex v is sum_a ((v_a - 1) mod 2) * 2^a. */
int vps_color_pass(vps_problem* p, int level, int prec, int mode, int color, const void* b, void* x);

/* r_coarse = P^T r_fine, P the embedding level-1 -> level (Sec. 2.1). fine_level >= 2. */
int vps_restrict(vps_problem* p, int fine_level, int prec, const void* r_fine, void* r_coarse);

/* vps_restrict without a problem object and without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same kernels and result as vps_restrict for (dim, degree, fine_level).
 * r_fine: device vector of n1d(fine_level)^dim values (boundary entries ignored); r_coarse:
 * device vector of n1d(fine_level - 1)^dim values (boundary entries written 0); FP64 when prec =
 * VPS_FP64, FP32 when VPS_FP32; both caller-owned.  hip_stream: the stream the launches go to
 * (NULL: the null stream); nothing synchronises.  The intermediate lives in a static device
 * array of 64 MiB per GPU held until the process ends, shared by every call on that GPU: calls
 * that overlap on one GPU race.  VPS_EINVAL when the intermediate (3D: n1d(fine)^2 *
 * n1d(fine-1) values of the precision's size; the 2D restriction has none) exceeds it, on a bad
 * shape or precision, or on a null vector; VPS_EHIP on a launch failure. */
int vps_restrict_noalloc(int dim, int degree, int fine_level, int prec, const void* r_fine, void* r_coarse,
                         void* hip_stream);

/* x_fine += P e_coarse (Sec. 2.1, Alg. 1 coarse-grid correction). fine_level >= 2. */
int vps_prolongate_add(vps_problem* p, int fine_level, int prec, const void* e_coarse, void* x_fine);

/* x = A_1^{-1} b on level 1 by one fast-diagonalisation patch solve, computed in FP64 for
 * both precisions (Sec. 2.1: one smoother step on the coarsest level is exact). */
int vps_coarse_solve(vps_problem* p, int prec, const void* b, void* x);

/* One V-cycle (Alg. 1) on the finest level, x in/out, 1 pre- and 1 post-smoothing step,
 * coarser levels start from 0; prec selects the V-cycle precision (the coarse solve is FP64).
 * Needs the matching VPS_FLAG_*_HIERARCHY. */
int vps_vcycle(vps_problem* p, int prec, const void* b, void* x);

/* Solve A x = b on the finest level by CG preconditioned with one V-cycle, from x = 0.
 * b, x: FP64 device vectors.  VPS_SOLVE_FP64: FP64 V-cycle, standard CG.
 * VPS_SOLVE_MIXED: the residual is rounded to FP32, one FP32 V-cycle (FP64 coarse solve)
 * approximates the error, the correction is widened to FP64; residuals, dot products and
 * updates stay FP64 (Sec. 4.2); CG uses the flexible (Polak-Ribiere) beta (also in FP64 mode
 * when the problem was created with VPS_FLAG_POST_SAME_ORDER).
 * Stops when ||r||_2 <= rtol ||b||_2.  Synchronises once per iteration; fills *stats
 * (may be NULL).  Returns VPS_OK, VPS_ENOCONV, VPS_EBREAKDOWN or VPS_ENOTFINITE. */
int vps_pcg_solve(vps_problem* p, int solve_mode, const double* b, double* x, double rtol, int maxit,
                  vps_solve_stats_t* stats);

/* Full multigrid (Alg. 2).  b_levels[l-1] (l = 1..L): device right-hand side of level l in
 * precision prec (boundary entries ignored); x: level-L result in prec (overwritten).
 * Level 1 is solved exactly, each finer level starts from the prolongated coarser solution
 * and takes one V-cycle; then V-cycles on level L repeat until ||b_L - A x||_2 <= eps ||b_L||_2
 * (interior norms) or maxit of them were taken.  stats->iterations counts those repeated
 * V-cycles (the n of Tables 1-2); rel_residual = true_rel_residual = the final ratio.
 * The colour order of the V-cycles follows VPS_FLAG_POST_SAME_ORDER.  Needs the matching
 * hierarchy flag and the solver vectors; synchronises once per V-cycle on level L.
 * Returns VPS_OK, VPS_ENOCONV or VPS_ENOTFINITE (stats filled in every case). */
int vps_fmg_solve(vps_problem* p, int prec, const void* const* b_levels, void* x, double eps, int maxit,
                  vps_solve_stats_t* stats);

/* b_i = int f phi_i for f = sum_m coef[m] prod_a sin(pi kappa[m*dim + a] x_a) on `level`
 * ((k+1)-point Gauss per cell direction; eq:matrix-def).  kappa, coef: host arrays. */
int vps_rhs_sine_modes(vps_problem* p, int level, int prec, int n_modes, const int* kappa,
                       const double* coef, void* b);

/* *err = || u - u_h ||_{L2(Omega)} for u = sum_m ucoef[m] prod_a sin(pi kappa[m*dim + a] x_a)
 * and u_h the FP64 finite element function with nodal values x (device, full level-`level`
 * grid), integrated cellwise with nq^d Gauss points (nq = 0: k+1; at most 16); the error
 * measure of the convergence study (Sec. 4.2, Table 7).  kappa, ucoef: host arrays.
 * Deterministic; synchronises the problem's stream. */
int vps_l2_error_sine_modes(vps_problem* p, int level, int n_modes, const int* kappa, const double* ucoef,
                            int nq, const double* x, double* err);

/* Wait for all work enqueued on the problem's stream. */
int vps_synchronize(vps_problem* p);

/* Message of the last failing call on this thread ("" if none). */
const char* vps_last_error(void);

/* Host-side check of the launch geometry of a hierarchy with fine level fine_level (no device
 * work; for tests and for callers sizing very large problems): on every level, every workgroup of
 * every colour pass (all colours, every launch shape the library uses) maps to patches of that
 * colour inside the grid, the workgroups cover each patch exactly once, and each workgroup's
 * farthest closure node is within the kernels' 32-bit byte offsets; every operator, restriction
 * and prolongation launch fits its launcher's limits (grid sizes, 32-bit offsets).  The patch
 * grid is the colouring of Sec. 2.2 (Fig. 2); the operator and transfers those of Secs. 2.1, 2.3.
 * *blocks_checked (may be NULL) receives the number of colour-pass workgroups enumerated.
 * VPS_OK, or VPS_EINVAL with the first violation in vps_last_error(). */
int vps_launch_geometry_check(int dim, int degree, int fine_level, long long* blocks_checked);

/* Host-side 1D tables for degree k (reference cell [0,1]) written to `out`, for tests:
 * which = 0: Gauss-Lobatto nodes (k+1); 1: reference stiffness (k+1)^2; 2: reference mass;
 * 3: patch eigenvectors S ((2k-1)^2, row-major, S^T M S = I, two-cell patch of unit cells);
 * 4: patch eigenvalues (2k-1); 5: prolongation coefficients ((2k+1) x (k+1)).
 * *n receives the value count; nothing is written when cap is too small. */
int vps_host_table(int k, int which, double* out, int cap, int* n);

/* ---- serving: continuous batching of Poisson solves (one GPU) ----------------
 * A server owns a device-memory budget.  Requests (dim, degree, level, rhs,
 * solve mode, tolerance) are queued on submit; vps_server_step advances every
 * admitted request by one CG iteration, packing the smoother colour passes of
 * requests that share (dim, degree, precision, level) into one launch, and
 * admits queued requests in arrival order whenever their footprint fits the
 * remaining budget and a slot is free.  Hierarchies are cached per (dim, degree,
 * level) and reused by later requests. */
typedef struct vps_server vps_server;

/* hbm_budget_bytes: device bytes the server may hold; max_active: concurrent requests.
 * hip_stream: the caller's stream (NULL: the null stream).  Each submit marks it, and the
 * request's first device work waits for that mark, so inputs written on this stream before
 * the submit are seen complete.  The server's own work runs on private streams. */
int vps_server_create(size_t hbm_budget_bytes, int max_active, void* hip_stream, vps_server** out);

/* Queue a request.  b_dev: FP64 rhs (device, N values, caller keeps it alive until done);
 * x_dev: FP64 output (device), valid once poll reports the request done (the server has then
 * waited for its last kernel; the caller must not touch x_dev before).  *ticket receives the
 * request id.  VPS_EBUSY if its footprint exceeds the whole budget; VPS_EHIP if the caller's
 * stream cannot be marked. */
int vps_server_submit(vps_server* s, int dim, int degree, int level, const double* b_dev, double* x_dev,
                      double rtol, int solve_mode, int maxit, long long* ticket);

/* One scheduler tick (admit, one CG iteration for every active request, retire). *n_active,
 * *n_queued (may be NULL) receive the counts after the tick.  Synchronises.  A request whose
 * launches fail finishes with the error code as its status (see poll) and returns its
 * hierarchy; the tick still returns VPS_OK and the server stays usable.  VPS_EHIP is returned
 * only when waiting on the device fails: every request in flight then ends with that status
 * and queued requests stay queued. */
int vps_server_step(vps_server* s, int* n_active, int* n_queued);

/* *done = 1 when the request finished (then *stats holds its result).  Host-only. */
int vps_server_poll(vps_server* s, long long ticket, int* done, vps_solve_stats_t* stats);

/* Tickets of requests finished since the previous call, in completion order: up to cap of them
 * are written to tickets (host array) and removed from the list, *n receives how many were
 * written.  Lets a caller with many requests in flight find completions without polling each
 * ticket.  Host-only; VPS_EINVAL on a null server or n, or on cap > 0 with a null array. */
int vps_server_completed(vps_server* s, long long* tickets, int cap, int* n);

/* Device bytes currently held by admitted requests and cached hierarchies. */
int vps_server_memory(vps_server* s, size_t* in_use, size_t* cached);

int vps_server_destroy(vps_server* s);

/* Testing hook for the failure paths of vps_server_step: the request `ticket` (not yet done)
 * has its next launch at `stage` (0: admission, 1: CG iteration, 2: preconditioner, which
 * ends its whole request group) report VPS_EHIP instead of running.  For callers that test
 * error handling without a faulty device; has no other effect.  VPS_EINVAL on an unknown or
 * finished ticket or a bad stage. */
int vps_server_inject_fault(vps_server* s, long long ticket, int stage);

#ifdef __cplusplus
}
#endif

#endif /* VPS_H */
