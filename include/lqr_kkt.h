/*
 * lqr_kkt.h -- C ABI of the MI355X (gfx950) LQR-KKT solver.
 *
 * The library solves, for a batch of independent instances, the
 * equality-constrained linear-quadratic subproblem that each primal-dual
 * iLQR / SQP iteration produces (Amatucci, Sousa-Pinto et al., arXiv
 * 2506.07823, Sec. II-B, eq. (QP)):
 *
 *   min  sum_{k<N} 1/2 x_k'Q_k x_k + 1/2 u_k'R_k u_k + x_k'M_k u_k + q_k'x_k + r_k'u_k
 *        + 1/2 x_N'Q_N x_N + q_N'x_N
 *   s.t. x_0 = x0,   x_{k+1} = A_k x_k + B_k u_k + c_k   (k = 0..N-1)
 *
 * and returns the primal solution (x, u) and the costates lam of the
 * Lagrangian of Sec. II-B (lam_0 multiplies x0 - x_0, lam_{k+1} multiplies
 * A_k x_k + B_k u_k + c_k - x_{k+1}), so that lam_k = P_k x_k + p_k with the
 * value function (P_k, p_k) of Sec. II-C.  M_k is the transpose of the paper's
 * cross-Hessian block S_k; c_k is the paper's affine dynamics term b_k; the
 * paper's stages i = 0..N with terminal N+1 are this ABI's k = 0..N-1 with
 * terminal N.
 *
 * Method (LQR_METHOD_SCAN): the value function is obtained by a reverse
 * parallel associative scan over conditional value functions (Sec. II-D,
 * eqs. (initialization) and (combination_rule)), the policy K_k, k_k in
 * parallel over stages (eq. (lqr)), the states by a parallel scan of the
 * closed-loop affine maps (eq. (controlled_dynamics)) and the costates by
 * lam_k = P_k x_k + p_k.  Depth is O(log N) combine levels instead of the N
 * dependent steps of the Riccati sweep.  LQR_METHOD_SEQ_RICCATI runs the
 * sequential Riccati recursion of Sec. II-C (one wavefront per instance); it
 * is the comparison baseline.
 *
 * Layout: every array is contiguous, row-major and batch-major, of the
 * dtype selected in lqr_opts (all arrays share it):
 *   A [batch][N][n][n]    B [batch][N][n][m]    c [batch][N][n]
 *   Q [batch][N+1][n][n]  R [batch][N][m][m]    M [batch][N][n][m]
 *   q [batch][N+1][n]     r [batch][N][m]       x0 [batch][n]
 *   x [batch][N+1][n]     u [batch][N][m]       lam [batch][N+1][n]
 *   status [batch] (int32)
 * Pointers must be device pointers (or pointers the device can access),
 * aligned to the element size.  Inputs are read-only; outputs may not alias
 * inputs or each other.
 *
 * Ownership: the caller allocates every input, output, status and the
 * workspace; the library never allocates or frees memory on the solve path.
 * A handle owns only its launch plans.  Calls are asynchronous on `stream`
 * (a hipStream_t; NULL selects the default stream): results are valid once
 * the stream has been synchronized.  A handle may be used by one host thread
 * at a time; concurrent solves on different streams need separate workspaces.
 *
 * Preconditions (documented, not silently regularized): R_k > 0, the stage
 * Schur complement Q_k - M_k R_k^{-1} M_k' >= 0 (> 0 for the scan's
 * Cholesky of the value function), Q_N > 0.  Then the KKT matrix is
 * nonsingular and every scan value matrix is positive definite.
 *
 * Errors: functions return LQR_OK (0) or a negative code; nothing is launched
 * when argument checking fails.  Per-instance numerical problems are
 * reported in `status` (bit flags below).  The call is asynchronous, so by
 * default it returns LQR_OK and the host learns of them after synchronizing
 * and reading `status`; with opts.sync_status set the call waits for the
 * stream, reads the status words and returns LQR_ENUMERIC if an instance
 * failed even after the FP64 fallback.
 *
 * FP64 fallback (FP32 calls, opts.fallback = 1): a Cholesky factorization of
 * the scan (R_k in the element, G_k in the policy, the value matrix and the
 * inner matrix of a combine; in the chunked schedule's sweeps at orders
 * 17..64 with m <= 16, where a leaf is combined through its rank-m factor
 * V = B R^{-1/2} by the Woodbury identity, the m x m matrix I + V' P V) with
 * a non-positive pivot or a condition
 * estimate (max L_ii / min L_ii)^2 above opts.cond_threshold marks its
 * instance; after the FP32 solve every marked instance is solved again whole
 * with FP64 arithmetic and FP64 intermediates (the sequential recursion of
 * eq. (lqr)), its FP32 outputs are overwritten, and its status carries bit 8.
 */
#ifndef LQR_KKT_H
#define LQR_KKT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define LQR_OK 0
#define LQR_EINVAL (-1)   /* bad size, null or misaligned pointer, bad option */
#define LQR_ENOMEM (-2)   /* workspace smaller than lqr_workspace_size reports */
#define LQR_ENUMERIC (-3) /* (opts.sync_status only) an instance failed even after the FP64 fallback */
#define LQR_EDEVICE (-4)  /* a HIP runtime call failed (see lqr_last_error) */
#define LQR_EUNSUPPORTED (-5) /* shape class not built into this library */

/* per-instance status bits (OR-ed) */
#define LQR_ST_NONFINITE 1    /* a non-finite value reached the output */
#define LQR_ST_NOT_SPD 2      /* R_k or G_k = R_k + B_k'P_{k+1}B_k not positive definite, even in FP64 */
#define LQR_ST_P_NOT_SPD 4    /* a scan value matrix lost positive definiteness */
#define LQR_ST_FP64_FALLBACK 8 /* the instance was solved again whole in FP64 (informational) */

typedef enum { LQR_F32 = 0, LQR_F64 = 1 } lqr_dtype;
typedef enum { LQR_METHOD_SCAN = 0, LQR_METHOD_SEQ_RICCATI = 1 } lqr_method;

typedef struct lqr_handle_s* lqr_handle_t;

typedef struct {
    int32_t dtype;          /* lqr_dtype of every array */
    int32_t method;         /* lqr_method */
    int32_t refine_sweeps;  /* iterative-refinement sweeps (scan method), 0..4: each computes the
                               FP64 KKT residual and, for the instances whose relative residual is
                               above refine_tol, re-solves the correction system with the factors
                               of the first solve (instances already within the tolerance are left
                               as they are).  Default: 1 for LQR_F32, 0 for LQR_F64. */
    int32_t fallback;       /* 1 (default): solve an instance again whole in FP64 when one of its FP32
                               factorizations fails or is ill-conditioned (see above) */
    double cond_threshold;  /* condition estimate above which the FP64 fallback fires (default 1e6) */
    double refine_tol;      /* relative KKT residual at or below which an instance is not refined
                               (default 1e-6: a tenth of the 1e-5 the FP32 path promises, so that an
                               instance is returned unrefined only well inside that tolerance) */
    double* resid_out;      /* optional device [batch] FP64: relative KKT residual of the returned
                               solution, ||r(x,u,lam)||_2 / ||(x0, c, q, r)||_2; NULL to skip */
    /* optional warm start (scan method; all three or none): device arrays in the layout and dtype
       of x, u, lam holding an initial solution, e.g. a stream's previous solve.  The factors are
       computed as usual; the returned solution is the warm one plus refinement corrections (at
       least one sweep), so the FP32 error scales with the distance from the warm start instead of
       with the solution.  They may be the output arrays themselves (updated in place); otherwise
       they must not overlap them.  NULL: cold start. */
    const void* warm_x;
    const void* warm_u;
    const void* warm_lam;
    int32_t sync_status;    /* 1: wait for the stream after the solve, read the status words and return
                               LQR_ENUMERIC if an instance has a failure bit (anything but bit 8);
                               not for use under stream capture.  Default 0 (asynchronous). */
} lqr_opts;

/* Fill *o with the defaults for `dtype` (scan method, refinement as above). */
void lqr_opts_default(lqr_opts* o, int32_t dtype);

/* Create a handle bound to HIP device `device`.  Returns LQR_OK,
 * LQR_EINVAL (null h, bad device) or LQR_EDEVICE. */
int lqr_create(lqr_handle_t* h, int device);

/* Destroy a handle (NULL is accepted). */
int lqr_destroy(lqr_handle_t h);

/* Bytes of device workspace lqr_kkt_solve needs for this problem shape;
 * opts may be NULL (defaults for LQR_F32).  A pure size computation: h may
 * be NULL and no device is touched. */
int lqr_workspace_size(lqr_handle_t h, int64_t batch, int N, int n, int m,
                       const lqr_opts* opts, size_t* bytes);

/* Solve `batch` independent instances (see the top of this file for the
 * problem, layout, ownership and error behaviour).  `workspace` is a device
 * buffer of at least lqr_workspace_size bytes, 256-byte aligned; its
 * contents need not be initialized and are clobbered.  `status` (device,
 * [batch]) receives the per-instance bit flags. */
int lqr_kkt_solve(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m,
                  const void* A, const void* B, const void* c, const void* Q,
                  const void* R, const void* M, const void* q, const void* r,
                  const void* x0, void* x, void* u, void* lam, int32_t* status,
                  void* workspace, size_t workspace_bytes, const lqr_opts* opts);

/* Re-solve with cached factors (the real-time-iteration pattern of Sec. II-F,
 * where successive subproblems of a stream often differ only in their
 * linear terms): same arguments as lqr_kkt_solve, where A, B, Q, R, M must be
 * the matrices of the last LQR_METHOD_SCAN lqr_kkt_solve of this shape on
 * this handle and this `workspace` (nothing else may have used it since),
 * and only x0, c, q, r may have changed.  The value function, policy and
 * closed-loop matrices that solve left in the workspace are reused: one
 * backward sweep of the gradient recursion of eq. (lqr) with the policy
 * fixed and one forward sweep per instance, O(N n^2) instead of O(N n^3),
 * then the FP64-residual refinement sweeps of opts (the matrices are read for
 * the residual).  On entry `status` must hold that solve's status words: an
 * instance with bit 8 (solved by the FP64 fallback) is solved again whole
 * in FP64, the others keep their bits.  Warm starts are not accepted. */
int lqr_kkt_resolve(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m,
                    const void* A, const void* B, const void* c, const void* Q,
                    const void* R, const void* M, const void* q, const void* r,
                    const void* x0, void* x, void* u, void* lam, int32_t* status,
                    void* workspace, size_t workspace_bytes, const lqr_opts* opts);

/* lqr_kkt_solve without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  The workspace is a fixed array
 * of lqr_noalloc_workspace_bytes() bytes (64 MiB) in the library's device
 * code, one per GPU, held until the process ends; its device address is
 * looked up once per device by lqr_create.  Nothing is allocated on this
 * path.  Arguments, layout, asynchrony and per-instance status are those of
 * lqr_kkt_solve.  Errors: LQR_ENOMEM (nothing launched) when the problem's
 * workspace (lqr_workspace_size) exceeds that size -- e.g. a single
 * whole-body instance (n=36, m=12, N=100) needs about 7 MB, so about eight
 * fit; LQR_EINVAL for opts->sync_status (it would allocate a host buffer)
 * and the argument errors of lqr_kkt_solve.  Every call on a GPU shares that
 * GPU's array and leaves its contents behind: calls that overlap on one GPU
 * (concurrent streams, several host threads) race and must be serialized by
 * the caller; successive calls on one stream are safe (no kernel reads
 * workspace contents it did not write in the same call). */
int lqr_kkt_solve_noalloc(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m,
                          const void* A, const void* B, const void* c, const void* Q,
                          const void* R, const void* M, const void* q, const void* r,
                          const void* x0, void* x, void* u, void* lam, int32_t* status,
                          const lqr_opts* opts);

/* Size of the workspace lqr_kkt_solve_noalloc uses (bytes, per GPU). */
size_t lqr_noalloc_workspace_bytes(void);

/* FP64 KKT residual of a given solution (x, u, lam) of the problem above:
 * writes rel[b] = ||r||_2 / ||(x0, c, q, r)||_2 per instance (device FP64
 * array).  The residual blocks are the stationarity conditions of the
 * Lagrangian of Sec. II-B plus the initial-condition and dynamics
 * constraints.  Uses `workspace` of lqr_workspace_size bytes. */
int lqr_kkt_residual(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m,
                     int32_t dtype, const void* A, const void* B, const void* c,
                     const void* Q, const void* R, const void* M, const void* q,
                     const void* r, const void* x0, const void* x, const void* u,
                     const void* lam, double* rel, void* workspace,
                     size_t workspace_bytes);

/* QP-data builder (the step before the solve, Sec. II-F): the blocks Q, M,
 * R, q, r of the subproblem from a nonlinear least-squares cost
 * 1/2 eps' W eps and relaxed barriers of constraints xi(x, u) >= 0, with the
 * Gauss-Newton approximation:
 *   Q = Ex' W Ex + Gx' D2 Gx,  M = Ex' W Eu + Gx' D2 Gu,  R = Eu' W Eu + Gu' D2 Gu,
 *   q = Ex' W eps + Gx' D1,    r = Eu' W eps + Gu' D1,
 * D1 = B'(xi), D2 = diag(B''(xi)) of the relaxed barrier
 *   B(xi) = -mu ln(xi) (xi >= delta), mu/2 (((xi - 2 delta)/delta)^2 - 1) - mu ln(delta) (xi < delta).
 * Inputs (device, dtype, row-major, batch-major): Ex [batch][N+1][p][n],
 * Eu [batch][N][p][m], e [batch][N+1][p] (eps at the linearization point),
 * W [batch][N+1][p][p], Gx [batch][N+1][nc][n], Gu [batch][N][nc][m],
 * g [batch][N+1][nc] (xi there), mu [nc], delta [nc] (per constraint, shared
 * by every instance and stage).  Outputs in the layout of lqr_kkt_solve's
 * Q, M, R, q, r.  nc may be 0 (the constraint arrays may then be NULL);
 * p (n + m) must fit one workgroup's LDS (64 KiB).  Asynchronous on
 * `stream`; needs no workspace. */
int lqr_qp_build(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m, int p, int nc, int32_t dtype,
                 const void* Ex, const void* Eu, const void* e, const void* W, const void* Gx, const void* Gu,
                 const void* g, const void* mu, const void* delta, void* Q, void* M, void* R, void* q, void* r);

/* SQP iteration around the solve (Sec. II-B, II-E, II-F) on a synthetic
 * nonlinear model with a bilinear dynamics term, standing in for the robot
 * models:
 *   h(x, u) = A x + B u + c + gamma (P x) .* (V u),
 *   stage cost 1/2 sum wx_k (x_k - xr_k)^2 + 1/2 sum wu_k (u_k - ur_k)^2
 *              + sum_j B(xi_j),  xi = Gx x + Gu u + g0 >= 0 (relaxed barrier
 *              of lqr_qp_build, parameters mu_j, delta_j),
 *   terminal cost without the control terms, initial state xhat0.
 * Arrays (device, call dtype, batch-major): A [batch][n][n], B [batch][n][m],
 * c [batch][n], P [batch][n][n], V [batch][n][m] (time-invariant per
 * instance), xr [batch][N+1][n], ur [batch][N][m], wx [batch][N+1][n],
 * wu [batch][N][m], Gx [batch][nc][n], Gu [batch][nc][m], g0 [batch][nc],
 * mu [nc], delta [nc], xhat0 [batch][n]. */
typedef struct {
    int64_t batch;
    int32_t N, n, m, nc;
    double gamma;
    const void *A, *B, *c, *P, *V, *xr, *ur, *wx, *wu, *Gx, *Gu, *g0, *mu, *delta, *xhat0;
} lqr_bilinear_model;

/* `iters` SQP iterations from the iterate (x [batch][N+1][n], u [batch][N][m],
 * lam [batch][N+1][n]; updated in place), each: linearize the dynamics and
 * the cost at the iterate (dynamics Jacobians, defects c_k = h(x_k, u_k) -
 * x_{k+1}, Gauss-Newton blocks by the QP-data builder), solve the
 * subproblem with lqr_kkt_solve's scan (opts: dtype, refinement, fallback,
 * mapping of the handle), then the parallel filter line search of Sec. II-E:
 * the ten trial steps alpha = 2^0 .. 2^-9 are evaluated at once (dynamics
 * violation theta = sum_k ||x_{k+1} - h(x_k, u_k)||_2 and cost, FP64
 * sums), and the largest accepted one is taken: with theta0 > theta_max
 * only a decrease of theta is accepted, else on a descent direction the
 * Armijo condition (eta 1e-4) on the cost, else a decrease of cost or
 * theta.  Update x += alpha dx, u += alpha du, lam += alpha (lam_QP - lam).
 * alpha_out (optional, [iters][batch]) receives the steps; a line search
 * that accepts none leaves the iterate and sets status bit 32.  status
 * ([batch]) holds the last iteration's solve status plus that bit.  n, m,
 * nc <= 64.  Workspace: lqr_sqp_workspace_size bytes, 256-byte aligned.
 * Asynchronous on `stream` (with opts->sync_status: LQR_ENUMERIC check at
 * the end). */
int lqr_sqp_workspace_size(lqr_handle_t h, int64_t batch, int N, int n, int m, int nc, const lqr_opts* opts,
                           size_t* bytes);
int lqr_sqp_solve(lqr_handle_t h, void* stream, const lqr_bilinear_model* mdl, int iters, double theta_max, void* x,
                  void* u, void* lam, void* alpha_out, int32_t* status, void* workspace, size_t workspace_bytes,
                  const lqr_opts* opts);
#define LQR_ST_LS_REJECTED 32   /* (lqr_sqp_solve) the line search accepted no step */

/* Diagnostics: the value function and policy of Sec. II-C that the last
 * LQR_METHOD_SCAN solve of this shape (same handle mapping, same workspace)
 * left in `workspace`: P [batch][N+1][n][n] and p [batch][N+1][n] (the
 * complete-suffix value functions P_k, p_k of the reverse scan), K
 * [batch][N][m][n] and kff [batch][N][m] (the policy of eq. (lqr)), device
 * arrays of the call's dtype.  Asynchronous on `stream`.  For an instance
 * that was solved again by the FP64 fallback (status bit 8) these are the
 * FP32 pass's values, not those of its returned solution. */
int lqr_kkt_factors(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m, int32_t dtype,
                    const void* workspace, size_t workspace_bytes, void* P, void* p, void* K, void* kff);

/* Diagnostics: while enabled, every kernel launch of lqr_kkt_solve /
 * lqr_kkt_residual on this handle is bracketed by two HIP events recorded on
 * the call's stream (adds two event records per launch).  Not for use under
 * stream capture. */
int lqr_timing_enable(lqr_handle_t h, int enable);

/* Waits for the recorded events and writes one text line per kernel family,
 * "name launches total_ms algorithmic_flops algorithmic_bytes", into buf
 * (NUL-terminated, at most len bytes), then forgets them.  The flops and
 * bytes are the algorithmic work of those launches (what the method must
 * compute and move, not what the padded tiles execute).  Returns
 * LQR_ENOMEM if buf is too small. */
int lqr_timing_report(lqr_handle_t h, char* buf, size_t len);

/* Mapping of a problem shape onto the GPU (for callers that want to pin it):
 *   engine   0 = default rule, 1 = wavefront tiles (orders <= 64, one 64-lane
 *            wavefront per task), 2 = matrix-core workgroups (one 256-thread
 *            workgroup per task, products on MFMA)
 *   fused    -1 = default (level by level), 0 = level-by-level launches of the
 *            vector-only passes, 1 = one workgroup per instance for them,
 *            2 = the whole solve (elements, scan, policy, forward scan,
 *            recovery, residual, refinement) in one launch, one workgroup
 *            of several wavefronts per instance (wavefront engine only)
 *   big_grid 0 = default (512), else the workgroups / scratch slots of a
 *            matrix-core task launch
 *   ms       (lqr_autotune output) mean time of one solve with this mapping
 *   split    schedule of the reverse scan (Sec. II-D; every schedule gives the
 *            same value functions, they differ in depth and work):
 *            0 = balanced tree over all N+1 scan elements (default);
 *            1 = split (wavefront engine, fused 0 or 1): the tree over the
 *            first 2^k elements (the largest power of two below N+1), the
 *            suffixes of the others by a sequential sweep of combines with
 *            the complete suffix to their right;
 *            2 = chunked (wavefront engine, fused 0 or 1): the last `sweep`
 *            elements by the sequential sweep, the others in chunks of
 *            `chunk` elements -- each chunk's aggregate by sequential
 *            combines, the complete suffixes at the chunk starts by a
 *            sequential pass over the aggregates, then the other suffixes
 *            of every chunk (chunk 1, or sweep N+1: the sequential
 *            information-form recursion)
 *   chunk    chunk length for split 2 (>= 1)
 *   sweep    elements of the sequential sweep for split 2 (1..N+1; the
 *            terminal element is always in it)
 *   fwd_seq  1 = forward scan, control/costate recovery and refinement
 *            vector passes as sequential sweeps over the stages (one task
 *            unit per instance, no forward-tree map products); fused 0 or 1
 *   streams  0 or 1 = the whole batch on the caller's stream; 2..4 = the
 *            batch in that many contiguous parts of ceil(batch / streams)
 *            instances, part 0 on the caller's stream and the others on
 *            side streams of the handle that wait for the work queued on
 *            the caller's stream before the call and that the caller's
 *            stream waits for after it (so the call stays asynchronous and
 *            stream-ordered, and can be captured into a graph).  The parts'
 *            launch sequences overlap on the GPU.  Each part has its own
 *            slice of the workspace; lqr_kkt_resolve and lqr_kkt_factors
 *            of the shape find the records in the same slices as long as
 *            the mapping is unchanged.  A handle's calls must not overlap
 *            (they share the side streams).  Ignored by the plain method. */
typedef struct {
    int32_t engine;
    int32_t fused;
    int32_t big_grid;
    float ms;
    int32_t split;
    int32_t chunk;
    int32_t sweep;
    int32_t fwd_seq;
    int32_t streams;
} lqr_tuning;

/* Pin (t != NULL) or clear (t == NULL) the mapping of the shape
 * (batch, N, n, m, dtype) on this handle; later lqr_workspace_size,
 * lqr_kkt_solve and lqr_kkt_residual calls of that shape use it.
 * LQR_EINVAL for an out-of-range field, engine 1 above order 64, fused 2
 * with the matrix-core engine, split 1 or 2 with the matrix-core engine or
 * fused 2, or fwd_seq with fused 2. */
int lqr_set_tuning(lqr_handle_t h, int64_t batch, int N, int n, int m, int32_t dtype, const lqr_tuning* t);

/* Autotuner: solves the given problem (same arguments as lqr_kkt_solve)
 * once per candidate mapping -- each engine that can take the shape, each
 * form of the passes (fused 0 / 1, fwd_seq 0 / 1, and the one-launch solve on
 * the wavefront engine), the reverse-scan schedules of the wavefront engine
 * (balanced tree, split, chunked with chunk 1 / 4 / 8 / 16 / 32 and a
 * one-element sweep), matrix-core grids of 256 / 512 / 1024
 * workgroups, and the three fastest of these again with the batch split
 * over 2 and 4 streams -- then `reps` more times on the stream, timed with
 * HIP events;
 * candidates whose status words are not clean (other than the FP64-fallback
 * bit) or whose workspace does not fit are skipped.  The fastest mapping is
 * stored on the handle for this shape (as lqr_set_tuning) and written to
 * *best.  Synchronizes the stream; the outputs hold the last candidate's
 * solution.  lqr_autotune_workspace_size gives a workspace that fits every
 * candidate.  Returns LQR_ENOMEM if no candidate fits. */
int lqr_autotune(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m,
                 const void* A, const void* B, const void* c, const void* Q, const void* R,
                 const void* M, const void* q, const void* r, const void* x0, void* x, void* u,
                 void* lam, int32_t* status, void* workspace, size_t workspace_bytes,
                 const lqr_opts* opts, int reps, lqr_tuning* best);
int lqr_autotune_workspace_size(int64_t batch, int N, int n, int m, const lqr_opts* opts, size_t* bytes);

/* Tuning cache.  lqr_autotune also records its choice per shape bucket
 * (dtype, n, m, N and batch rounded up to powers of two), and a solve of a
 * shape with no exact mapping pinned uses its bucket's.  lqr_tuning_save
 * writes the buckets of this handle to a text file at `path` (replacing the
 * entries of this device's architecture, keeping those of others);
 * lqr_tuning_load reads the entries of this device's architecture into the
 * handle and returns how many it loaded (>= 0), or LQR_EINVAL if the file
 * cannot be read. */
int lqr_tuning_save(lqr_handle_t h, const char* path);
int lqr_tuning_load(lqr_handle_t h, const char* path);

/* One problem of a ragged batch: its sizes and the device arrays of one
 * instance in the layout above (without the batch axis). */
typedef struct {
    int32_t N, n, m, reserved;
    const void *A, *B, *c, *Q, *R, *M, *q, *r, *x0;   /* inputs */
    void *x, *u, *lam;                                /* outputs */
} lqr_problem;

/* Ragged batch: `count` independent problems of mixed (N, n, m) in one call
 * (the equality-constrained LQ subproblem of Sec. II-B for each).  The
 * host-side descriptor table `probs` is read during the call only.  Problems
 * of one shape are gathered into a contiguous batch in the workspace
 * (packing kernels), solved together exactly as lqr_kkt_solve solves a
 * batch (so each result equals that of solving the problem alone), and
 * scattered back; shapes run one after another on `stream`.  status
 * (device [count]) and opts->resid_out (optional device [count]) are in
 * descriptor order.  Warm starts are not accepted here.  The workspace must
 * hold lqr_ragged_workspace_size bytes (the largest shape group's packed
 * arrays and solve workspace).  Errors as lqr_kkt_solve; a bad descriptor
 * makes the call return LQR_EINVAL before any launch. */
int lqr_ragged_workspace_size(lqr_handle_t h, int64_t count, const lqr_problem* probs, const lqr_opts* opts,
                              size_t* bytes);
int lqr_kkt_solve_ragged(lqr_handle_t h, void* stream, int64_t count, const lqr_problem* probs,
                         int32_t* status, void* workspace, size_t workspace_bytes, const lqr_opts* opts);

/* Ragged batch from a device descriptor table (persistent form).  Problem
 * i is described by descs[i] (device memory, read by the kernels): its sizes,
 * the element offsets of its nine input arrays (A, B, c, Q, R, M, q, r, x0, in
 * the per-instance layout above) in the packed input buffer `in`, the
 * offsets of its outputs (x, u, lam) in the packed output buffer `out`, and
 * status_idx, the index of its status word (and residual, opts->resid_out)
 * in [0, count).  Every problem is solved whole -- scan elements, reverse
 * scan, policy, forward scan, recovery, FP64 residual and refinement sweeps
 * (Sec. II-C / II-D) -- by one workgroup of a persistent kernel per padded
 * order class (orders up to 64): `slots` workgroups, each with one workspace
 * slot sized for N <= maxN and n, m <= maxd, take the problems from an
 * atomic counter, so problems of any mix of shapes share launches and the
 * host never reads the table.  Problems marked for the FP64 fallback are
 * then solved again whole in FP64.  The call is asynchronous on `stream`
 * and can be captured into a graph and replayed with new table and buffer
 * contents (a descriptor with N = 0 marks an unused entry of a fixed-size
 * table).  A descriptor with malformed sizes (N = 0 included), n or m above
 * 64 or shapes beyond (maxN, maxd) is not solved: its status word gets
 * LQR_ST_BAD_DESC and its residual -1; a descriptor whose status_idx is out
 * of range is ignored.  opts->warm_x/u/lam, when given, are packed buffers laid
 * out like `out` (every problem warm-started).  The workspace must hold
 * lqr_ragged_dev_workspace_size bytes (proportional to slots, not count),
 * 256-byte aligned. */
typedef struct {
    int32_t N, n, m, status_idx;
    int64_t in_off[9];    /* A, B, c, Q, R, M, q, r, x0 (elements into `in`) */
    int64_t out_off[3];   /* x, u, lam (elements into `out`) */
} lqr_problem_desc;
#define LQR_ST_BAD_DESC 16   /* ragged descriptor malformed or beyond the slots (not solved) */

int lqr_ragged_dev_workspace_size(int64_t count, int32_t slots, int32_t maxN, int32_t maxd, const lqr_opts* opts,
                                  size_t* bytes);
int lqr_kkt_solve_ragged_dev(lqr_handle_t h, void* stream, int64_t count, const lqr_problem_desc* descs,
                             const void* in, void* out, int32_t* status, int32_t slots, int32_t maxN, int32_t maxd,
                             void* workspace, size_t workspace_bytes, const lqr_opts* opts);

/* Largest n, m supported by the built shape classes (n, m <= this). */
int lqr_max_dim(void);

/* Message describing the last error returned on this host thread. */
const char* lqr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LQR_KKT_H */
