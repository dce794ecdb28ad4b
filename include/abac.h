/* abac.h -- C ABI of the MI355X (gfx950) ABAC-preconditioned MINRES wave solver.
 *
 * The library solves the time-reversed all-at-once system Y T u = Y f of the
 * implicit leap-frog discretisation of u_tt = Laplace(u) + f on (0,1)^d, d = 1, 2,
 * with homogeneous Dirichlet data (Lin & Hon, Section 1, eqs. (1.1)-(1.4)), by
 * MINRES preconditioned with the absolute-value block alpha-circulant matrix
 * P_alpha = (C_alpha^{1/2})^T C_alpha^{1/2} (eqs. (1.5)-(1.10); fast apply in
 * Section 2.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Grid: nx interior points in x (h = 1/(nx+1)); ny interior points in y, or
 *   ny = 0 for the 1D problem; nt time levels, tau = T/nt.  Supported sizes:
 *   nx+1 a power of two in [8, 4096] (1D) or [8, 512] (2D); ny+1 a power of two in
 *   [8, 512] (2D); nt a power of two in [8, 1024].  Other sizes give ABAC_EINVAL.
 * - Vectors are FP64 DEVICE pointers owned by the caller, laid out
 *   [batch][nt][ny][nx] with x fastest (ny omitted in 1D); one vector holds
 *   N = nt * nx * max(ny,1) values per right-hand side.  Level k (0-based) of a
 *   solution vector is u^(k+1) of eq. (1.2).  Pointers must be 8-byte aligned and
 *   must not alias unless stated.
 * - Every call is asynchronous on the plan's HIP stream unless stated otherwise.
 * - Calls return an abac_status and never throw; abac_last_error() returns a
 *   thread-local description of the last failure.
 * - A plan is bound to one stream and is not thread-safe; distinct plans are
 *   independent and may run concurrently on different streams.
 */
#ifndef ABAC_H
#define ABAC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct abac_plan abac_plan;

typedef enum {
  ABAC_OK = 0,
  ABAC_EINVAL = -1,      /* bad argument or unsupported size                          */
  ABAC_ENOMEM = -2,      /* device allocation failed or workspace too small           */
  ABAC_EDEVICE = -3,     /* a HIP runtime call failed                                 */
  ABAC_ENOTCONV = -4,    /* MINRES did not reach tol within maxit (last iterate kept) */
  ABAC_EBREAKDOWN = -5,  /* <q, P^{-1} q> <= 0 or non-finite (e.g. NaN/Inf input)     */
  ABAC_EBUDGET = -6,     /* server: request larger than the whole memory budget       */
  ABAC_EAGAIN = -7       /* server: result not ready yet                              */
} abac_status;

typedef enum {
  ABAC_PREC_FP64 = 0,    /* every transform of the preconditioner in FP64             */
  ABAC_PREC_FP32 = 1,    /* preconditioner transforms in FP32 complex; the Krylov
                            recurrences, inner products and residual stay FP64        */
  ABAC_PREC_NONE = 2     /* no preconditioner (P = I): plain MINRES, the comparison
                            solver "MINRES-I" of Section 3; alpha is ignored           */
} abac_prec;

/* Bytes of device workspace a plan with these parameters needs (0 if invalid).
 * batch = number of right-hand sides the plan processes per call (>= 1). */
size_t abac_workspace_bytes(int nx, int ny, int nt, int prec, int batch);

/* Create a plan for the grid (nx, ny, nt), final time T > 0 and alpha in (0, 1]
 * (alpha = 1 is the absolute-value block circulant of the remark after eq. (1.10);
 * alpha in (0,1) the ABAC preconditioner).  The spectral tables (DST eigenvalues
 * of the Laplacian, alpha^{t/nt} scalings, FFT twiddles) are computed in FP64 on
 * the host and copied into the workspace.
 *   stream:      a hipStream_t (NULL = default stream); all work is enqueued there.
 *   workspace:   device memory of at least abac_workspace_bytes(...) bytes owned by
 *                the caller for the plan's lifetime, or NULL to let the library
 *                allocate (and free at destroy) its own.
 * Host-synchronous with respect to its table upload.  *out is set on success. */
abac_status abac_plan_create(int nx, int ny, int nt, double T, double alpha, int prec, int batch,
                             void *stream, void *workspace, size_t workspace_bytes, abac_plan **out);

/* Workgroup sizes (threads) of the plan's transform kernels, wg[0..4]:
 * wg[0] first x-DST pass, wg[1] y-DST pass, wg[2] time pass, wg[3] last x-DST pass,
 * wg[4] the fused x-y first and last passes, or 0 where the plan uses the separate
 * passes.  The fused passes serve square 2D grids whose whole level fits in LDS: one
 * workgroup per time level applies both spatial DSTs (Section 2.3's fast sine
 * transforms) there, so the y passes over memory disappear; their tile follows a fixed
 * rule of the shape (ABAC_SLAB=0 in the environment keeps the separate passes).  wg[5] is 512 when
 * small 1D problems (nt * nx <= 4096) run each MINRES iteration as one launch, one
 * 512-thread workgroup per right-hand side doing every step in turn (launch latency,
 * not memory, bounds the separate kernels there; ABAC_SMALL=0 keeps them), else 0.  The other tiles are
 * chosen by a tuner that times every legal tile on the plan's own buffers at creation
 * and caches the choice per shape (ABAC_TUNE=0 keeps 256-thread defaults;
 * ABAC_TUNE_FILE names an optional cache file).  wg must hold 6 ints. */
abac_status abac_plan_tiles(abac_plan *plan, int *wg);

/* Override the tiles the tuner chose for the plan's first x-DST pass (wg_x), y-DST pass
 * (wg_y, 2D only), time pass (wg_t) and last x-DST pass (wg_xi), in threads per
 * workgroup; 0 keeps the current choice.  Every sequence of the fast transforms of
 * Section 2.3 is computed by the same arithmetic whatever the tile, and the one
 * reduction these passes carry in a MINRES solve (the time pass's partials of
 * <q, P^{-1} q>) is summed in an order fixed by the sequence length, so every legal tile
 * gives bitwise the same results; this call lets a caller (a test) run each one.
 * ABAC_EINVAL (nothing changed) if a tile is not legal for its kernel (it must be a
 * multiple of 64 and of the threads per sequence, and its LDS must fit the device), if
 * the plan uses the fused x-y passes and wg_x, wg_y or wg_xi is nonzero, for
 * ABAC_PREC_NONE, or while a solve is in progress.  Synchronises the plan stream. */
abac_status abac_plan_set_tiles(abac_plan *plan, int wg_x, int wg_y, int wg_t, int wg_xi);

/* Release the plan (synchronises its stream; frees library-owned memory only). */
abac_status abac_plan_destroy(abac_plan *plan);

/* Variable coefficient of the wave equation u_tt = div(a grad u) + f (Section 3,
 * eq. (3.1)).  Afterwards the matrix-vector product, the right-hand side and the
 * explicit residual use L_a = I - (tau^2/2) Delta_{a,h} (eq. (3.2)), the conservative
 * central difference (a_e (u_e - u) - a_w (u - u_w))/hx^2 + (same in y)/hy^2 with a
 * taken at the cell faces; the preconditioner is built from the mean-coefficient
 * matrix with L_abar = I - (abar tau^2/2) Delta_h (eq. (3.3)).
 *   a_xh:  HOST array [ny1][nx+1] (ny1 = max(ny,1)): a at (x_{i+1/2}, y_j),
 *          x_{i+1/2} = (i + 1/2) hx for i = 0..nx, y_j = (j+1) hy (row 0 in 1D);
 *   a_yh:  HOST array [ny+1][nx] (2D only; ignored in 1D): a at (x_i, y_{j+1/2});
 *   abar:  the preconditioner's constant coefficient (the paper takes the mean of a
 *          over the grid points), > 0.
 * a_xh = NULL restores the constant coefficient a = 1 (abar ignored).  Every entry
 * must be positive and finite (ABAC_EINVAL otherwise, nothing changed).  The face
 * weights are copied into the workspace; host-synchronous; not allowed while a
 * solve is in progress (ABAC_EINVAL). */
abac_status abac_plan_set_coefficient(abac_plan *plan, const double *a_xh, const double *a_yh, double abar);

/* Right-hand side f of eq. (1.2) from source samples src = f^(0..nt-1)
 * ([batch][nt][...]), initial displacement psi0 and velocity psi1 ([batch][...],
 * one level each):  f_1 = tau^2 f^(0)/2 + tau psi1 + psi0,
 * f_2 = tau^2 f^(1) - L psi0,  f_k = tau^2 f^(k-1) for k >= 3,
 * with L = I - (tau^2/2) Laplace_h (L_a with a variable coefficient, eq. (3.2)).
 * f must not alias the inputs. */
abac_status abac_build_rhs(abac_plan *plan, const double *src, const double *psi0, const double *psi1,
                           double *f);

/* y = Y T x (eqs. (1.2), (1.4)): (T x)^(k) = L (x^(k) + x^(k-2)) - 2 x^(k-1), stored
 * at level nt-1-k.  y must not alias x. */
abac_status abac_apply_A(abac_plan *plan, const double *x, double *y);

/* y = T x (eq. (1.2)) in natural time order (no reversal): (T x)^(k) = L (x^(k) +
 * x^(k-2)) - 2 x^(k-1) (L_a with a variable coefficient).  y must not alias x. */
abac_status abac_apply_T(abac_plan *plan, const double *x, double *y);

/* z = C_alpha^{-1} r: the block alpha-circulant preconditioner itself (eqs.
 * (1.5)-(1.7), the matrix of the prior work the paper starts from), computed as
 * S [D^{-1} F^{-1} diag(mu^{-1}) F D] S: one spatial DST pair and one time FFT pair per
 * mode, no time reversal.  With ABAC_PREC_NONE, z = r.  z may alias r.  Not allowed while
 * a solve is in progress (ABAC_EINVAL). */
abac_status abac_apply_Cinv(abac_plan *plan, const double *r, double *z);

/* z = P_alpha^{-1} r = C_alpha^{-1/2} (C_alpha^{-1/2})^T r (eq. (1.9), Section 2.3),
 * computed as S [K Y K Y] S with S the orthonormal DST-I in space and
 * K = D^{-1} F^{-1} diag(mu^{-1/2}) F D per spatial mode in time (the transposed
 * factor uses (C^{-1/2})^T = Y C^{-1/2} Y).  z may alias r. */
abac_status abac_apply_Pinv(abac_plan *plan, const double *r, double *z);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): z = P_alpha^{-1} r as abac_apply_Pinv
 * computes it, for `batch` right-hand sides of the grid (nx, ny, nt) with final time T,
 * alpha and transform precision prec (ABAC_PREC_FP64 or ABAC_PREC_FP32), without a
 * plan.  It calls no hipMalloc, hipFree or other allocating routine: the spectral
 * tables (computed on the device) and the transform scratch live in a fixed device
 * array of 128 MiB inside the library, one per GPU, held until the process ends.
 *   r, z:    caller-owned DEVICE vectors [batch][nt][...], FP64; z may alias r.
 *   stream:  hipStream_t (NULL = default stream); the call is asynchronous on it.
 * Sizes, tiles and results follow abac_apply_Pinv's rules (the tuned tiles of a plan are
 * replaced by the tuner's default tiles; the passes carry no reduction, so the result
 * is the same).  ABAC_EINVAL if the tables plus batch * nt * (nx+1) * max(ny,1)
 * transform values (8 bytes each in FP64, 4 in FP32) exceed 128 MiB, if alpha is not
 * in (0, 0.5] (near 1 C_alpha can be singular; a plan checks that), or for
 * ABAC_PREC_NONE.  Every call on one GPU uses that GPU's single array: calls that
 * overlap on one GPU (different streams or threads without ordering) race and give
 * wrong results; calls ordered on one stream are safe. */
abac_status abac_apply_Pinv_noalloc(int nx, int ny, int nt, double T, double alpha, int prec, int batch,
                                    const double *r, double *z, void *stream);

/* Solve Y T u = Y f for every right-hand side in the batch by preconditioned MINRES
 * with zero initial guess (Section 3).  Stops a right-hand side at the first
 * iteration whose residual ||Y f - Y T u||_2 <= tol ||Y f||_2 (tracked by the MINRES
 * residual recurrence and confirmed explicitly; iterations continue with explicit
 * checks if the confirmation fails).  Host-synchronous.  f must stay valid and
 * unchanged during the call; u receives the iterates.
 *   iters, relres, status: host arrays of length batch (status may be NULL) that
 *   receive per right-hand side the iteration count, the explicit relative residual
 *   and the status (ABAC_OK, ABAC_ENOTCONV with the last iterate in u, or
 *   ABAC_EBREAKDOWN).
 * Returns ABAC_OK if every right-hand side converged, otherwise the first failing
 * status. */
abac_status abac_minres_solve(abac_plan *plan, const double *f, double *u, double tol, int maxit,
                              int *iters, double *relres, int *status);

/* Asynchronous form of abac_minres_solve for overlapping solves on several plans:
 * begin() enqueues the set-up, advance(k) enqueues k more iterations (right-hand
 * sides that have stopped skip their work on the device), poll() reports without
 * blocking whether every right-hand side of the plan has stopped as of the last
 * completed poll point (*done = 1) and finish() waits and fills the per-RHS results
 * like abac_minres_solve. */
abac_status abac_minres_begin(abac_plan *plan, const double *f, double *u, double tol, int maxit);
abac_status abac_minres_advance(abac_plan *plan, int iterations);
abac_status abac_minres_poll(abac_plan *plan, int *done);
abac_status abac_minres_finish(abac_plan *plan, int *iters, double *relres, int *status);

/* ---------------------------------------------------------------------------
 * Groups: solves of different grids advanced together.  A group holds up to 64 plans
 * (any mix of 1D and 2D grids, batches, alphas and final times; one transform
 * precision), each with a solve begun by abac_minres_begin.  abac_group_advance runs
 * one MINRES iteration (Section 3's solver) of every member with ONE launch per step
 * of the iteration for all of them -- the matvec, the scalar steps, the three
 * transform passes of Section 2.3 done twice, the residual recurrence and the
 * stopping test -- instead of one launch per step per member, which is what bounds
 * small grids.  Each member's results are bitwise those of its own solve
 * (abac_minres_solve on the same plan): the same tiles compute the same values and
 * every reduction is grouped as in the member's own kernels.
 * ------------------------------------------------------------------------- */
typedef struct abac_group abac_group;

/* Create an empty group whose launches go to `stream` (a hipStream_t, NULL = the
 * default stream).  Allocates a small device table (hipMalloc). */
abac_status abac_group_create(void *stream, abac_group **out);

/* Release the group (synchronises its stream); the member plans are not touched. */
abac_status abac_group_destroy(abac_group *group);

/* Set the members: n plans (0 <= n <= 64, no plan twice), each with a solve in progress
 * (abac_minres_begin), the same transform precision (ABAC_PREC_FP64 or ABAC_PREC_FP32)
 * and not on the one-launch small-problem path (abac_plan_tiles wg[5] = 0); a member's
 * transform lengths must have 256-thread tiles (1D grids up to nx = 2047).  The
 * group's stream waits for each member's stream (its set-up).  The plans' state is
 * copied: a member must not be changed (abac_plan_set_coefficient, abac_plan_set_tiles)
 * or advanced on its own while it is in the group.  ABAC_EINVAL otherwise.  The new
 * membership takes effect in stream order: launches already enqueued keep the old one.
 * A member that leaves must be finished (abac_minres_finish) before it is changed. */
abac_status abac_group_set(abac_group *group, abac_plan *const *plans, int n);

/* Enqueue `iterations` MINRES iterations of every member (members that have stopped
 * skip their work on the device), then make every member's stream wait for them.
 * Afterwards abac_minres_poll and abac_minres_finish work on each member as after
 * abac_minres_advance. */
abac_status abac_group_advance(abac_group *group, int iterations);

/* The same `iterations` MINRES iterations of every member as abac_group_advance, with
 * bitwise the same results, in ONE persistent launch of `blocks` 256-thread workgroups
 * (0: a default that balances barrier cost against parallelism; always capped at what
 * the device holds at once and at the largest step's logical blocks), each taking
 * every gridDim-th logical block of a step, with a grid-wide barrier between steps.
 * Other work on the device can only delay the launch (its blocks become resident as
 * that work ends).  Every block's barrier writes back and invalidates its XCD's
 * L2 (agent scope), so a barrier costs more per block than a launch costs per step:
 * the persistent launch suits groups of small grids run on few blocks.  A block that
 * waits longer than timeout_s seconds at a barrier (0: 2 s) leaves the launch, and so
 * do the others: the launch still ends, but the members' state is then invalid and
 * abac_group_check reports it.  The device current at abac_group_create must be
 * current.  Asynchronous as abac_group_advance; ABAC_EINVAL for an argument out of
 * range or another current device, ABAC_EDEVICE if the device refuses the launch. */
abac_status abac_group_run(abac_group *group, int iterations, int blocks, double timeout_s);

/* Wait for the group's stream; *aborted = 1 if a persistent launch (abac_group_run)
 * stopped waiting at a barrier since the last check, else 0.  Clears the flag. */
abac_status abac_group_check(abac_group *group, int *aborted);

/* Restarted GMRES(restart) for the non-symmetric system T u = f with right
 * preconditioning by C_alpha (the block alpha-circulant preconditioner, which is not
 * symmetric and so needs a non-symmetric Krylov solver), x_0 = 0.  Stops at the first
 * step whose rotated residual ||f - T u||_2 (equal to the true residual with right
 * preconditioning) is <= tol ||f||_2, confirmed explicitly; a cycle of `restart` steps
 * ends by forming u and restarting from its explicit residual.  f, u: [batch][nt][...]
 * device vectors (u must not alias f); iters, relres, status: host arrays of batch
 * entries (may be NULL).  1 <= restart <= 15 (the Arnoldi basis uses the plan's Krylov
 * vectors).  Host-synchronous (one small device-to-host read per step).  Returns
 * ABAC_OK, ABAC_ENOTCONV (some right-hand side reached maxit), ABAC_EBREAKDOWN
 * (non-finite values) or ABAC_EINVAL. */
abac_status abac_gmres_solve(abac_plan *plan, const double *f, double *u, double tol, int maxit, int restart,
                             int *iters, double *relres, int *status);

/* Kernel-time accounting (for roofline reports).  When enabled, every kernel the
 * plan launches is bracketed by HIP events on the plan stream.  read() synchronises
 * the stream and returns, for kernel class k (see ABAC_K_*), the summed duration in
 * milliseconds and the number of launches since the last reset. */
enum {
  ABAC_K_STENCIL = 0,   /* Y T x matvec (and the fused <A z, z>)        */
  ABAC_K_DSTX_FWD = 1,  /* first spatial DST pass (x)                   */
  ABAC_K_DSTY = 2,      /* y-direction DST pass (2D, both directions)   */
  ABAC_K_TIME = 3,      /* per-mode time pipeline K Y K Y               */
  ABAC_K_DSTX_INV = 4,  /* last spatial DST pass (x)                    */
  ABAC_K_UPDATE = 5,    /* MINRES residual (and late w / x) update      */
  ABAC_K_RESIDUAL = 6,  /* explicit residual check                      */
  ABAC_K_INIT = 7,      /* solve set-up                                 */
  ABAC_K_RHS = 8,       /* right-hand side assembly                     */
  ABAC_K_FIN = 9,       /* per-RHS scalar steps (sums of partials)      */
  ABAC_K_FORM = 10,     /* stopping test; iterate from the resident basis */
  ABAC_K_GMRES = 11,    /* GMRES vector kernels (dots, axpys, scalings)  */
  ABAC_K_ITER = 12,     /* whole iteration in one workgroup per RHS (small 1D problems) */
  ABAC_K_COUNT = 13
};
abac_status abac_profile_enable(abac_plan *plan, int on);
abac_status abac_profile_read(abac_plan *plan, int kernel, double *total_ms, long long *launches);
abac_status abac_profile_reset(abac_plan *plan);

/* Fill out[0..n) (DEVICE pointer) with i.i.d. N(0,1) values from the counter-based
 * Philox4x32-10 generator keyed by `seed` (element e: counter e/4; the four words
 * become two Box-Muller pairs), on `stream`.  Used for seeded synthetic sources. */
abac_status abac_fill_normal(void *stream, double *out, size_t n, unsigned long long seed);

/* ---------------------------------------------------------------------------
 * Request server (continuous batching).  Requests of any supported shape are queued,
 * admitted while their device memory (plan workspace + right-hand side + solution)
 * fits an HBM byte budget and a cap on concurrent solves, and advanced one MINRES
 * iteration at a time on their own HIP streams, so solves admitted at different
 * times overlap on the device.  Finished solves free their slot at once; plans and
 * buffers of idle slots are cached per shape and evicted (least recently used) when
 * a new request needs the memory.  A request's source is i.i.d. N(0,1)
 * (abac_fill_normal with its seed) with zero initial data.  Not thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct abac_server abac_server;

abac_status abac_server_create(size_t budget_bytes, int max_active, abac_server **out);
abac_status abac_server_destroy(abac_server *server);

/* Group lane: requests whose right-hand side has at most max_unknowns unknowns (and
 * whose grid a group accepts, see abac_group_set) run as members of one group on a
 * stream of the server's own, so a step advances all of them with one launch per
 * MINRES step; the others keep their own streams.  0 (the default) turns the lane off.
 * Lane members do not count against max_active (the lane holds up to 64 of them).
 * Only while the server is idle (no request queued or active): ABAC_EINVAL otherwise.
 * Results are the same either way (bitwise). */
abac_status abac_server_group_lane(abac_server *server, size_t max_unknowns);

/* Queue a solve of grid (nx, ny, nt), final time T, alpha, preconditioner precision
 * prec, to relative residual tol within maxit iterations.  arrival_s is the arrival
 * time on the server clock (abac_server_clock); latency is measured from it.  With
 * keep_solution != 0 the solution stays on the device until abac_server_result
 * copies it out.  ABAC_EBUDGET if the request can never fit the budget. */
abac_status abac_server_submit(abac_server *server, int nx, int ny, int nt, double T, double alpha, int prec,
                               unsigned long long seed, double tol, int maxit, double arrival_s, int keep_solution,
                               long long *ticket);

/* Make progress without blocking: admit what fits, queue iterations, retire finished
 * solves.  *active / *queued (may be NULL) receive the current counts. */
abac_status abac_server_step(abac_server *server, int *active, int *queued);

/* ABAC_EAGAIN while the request is pending.  Otherwise fills iters, relres, status,
 * latency_s (arrival to observed completion) and, if u_host != NULL and the request
 * kept its solution, copies the N solution values to host memory; then forgets the
 * ticket.  Any pointer argument may be NULL. */
abac_status abac_server_result(abac_server *server, long long ticket, double *u_host, int *iters, double *relres,
                               int *status, double *latency_s);

/* Seconds since the server was created. */
double abac_server_clock(abac_server *server);

/* Device bytes currently held by the server (active and cached idle slots). */
size_t abac_server_bytes_in_use(abac_server *server);

/* Constant string for a status code. */
const char *abac_status_string(int status);

/* Thread-local description of the last error ("" if none). */
const char *abac_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ABAC_H */
