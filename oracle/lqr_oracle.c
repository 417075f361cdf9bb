/*
 * lqr_oracle.c -- CPU FP64 oracle for the LQR KKT solve of primal-dual iLQR
 * (Amatucci, Sousa-Pinto et al., "Primal-Dual iLQR for GPU-Accelerated
 * Learning and Control in Legged Robots", arXiv 2506.07823).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * never links, loads or calls it, and it shares no code with the GPU path.
 *
 * Everything here is plain, slow, obviously correct double precision code:
 * naive triple loops, a textbook Cholesky, Gaussian elimination with partial
 * pivoting.  No blocking, no fusion, no reordering beyond the equations.
 *
 * Conventions (fixed once for the whole project; the paper's own indices
 * drift between the OCP and the QP statement):
 *   N stages k = 0..N-1 with a terminal node k = N.
 *   x_k in R^n (k = 0..N), u_k in R^m (k = 0..N-1), lambda_k in R^n (k=0..N).
 *   Stage cost  1/2 x'Q_k x + 1/2 u'R_k u + x'M_k u + q_k'x + r_k'u,
 *   i.e. the paper's Hessian block [[Q, S'],[S, R]] with S_k = M_k' (m x n).
 *   Terminal cost 1/2 x'Q_N x + q_N'x.
 *   Dynamics  x_{k+1} = A_k x_k + B_k u_k + c_k  (c_k is the paper's b_k),
 *   initial condition x_0 = x0.
 *   All matrices row-major, contiguous, stage-major:
 *     A[N][n][n] B[N][n][m] c[N][n] Q[N+1][n][n] R[N][m][m] M[N][n][m]
 *     q[N+1][n] r[N][m] x0[n];  x[N+1][n] u[N][m] lam[N+1][n].
 *
 * Functions and the passages they follow:
 *   lqro_riccati          Sec. II-C, eq. (lqr) backward recursion, forward
 *                         pass and costate update delta-lambda = P dx + p.
 *   lqro_riccati_batch    the same, over independent instances (pthreads).
 *   lqro_kkt_residual     Sec. II-B, stationarity of the Lagrangian together
 *                         with the initial-condition and dynamics constraints.
 *   lqro_element          Sec. II-D, eq. (initialization): the conditional
 *                         value function of one stage in dual form.
 *   lqro_combine          Sec. II-D, eq. (combination_rule), read with the
 *                         corrections listed at the function.
 *   lqro_affine_combine   Sec. II-D, composition of conditional optimal
 *                         trajectories, eq. (conditional_optimal_trajectory),
 *                         read with the order correction at the function.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small dense helpers (row-major)                                    */
/* ------------------------------------------------------------------ */

/* C[r x c] = op(X) * op(Y); tx/ty select transposition of the operand as
 * stored.  X stored as (tx ? k x r : r x k), Y stored as (ty ? c x k : k x c). */
static void mm(int r, int c, int k, const double* X, int tx, const double* Y,
               int ty, double* C) {
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) {
            double s = 0.0;
            for (int l = 0; l < k; ++l) {
                double xv = tx ? X[l * r + i] : X[i * k + l];
                double yv = ty ? Y[j * k + l] : Y[l * c + j];
                s += xv * yv;
            }
            C[i * c + j] = s;
        }
}

/* y[r] = op(X) * v */
static void mv(int r, int k, const double* X, int tx, const double* v,
               double* y) {
    for (int i = 0; i < r; ++i) {
        double s = 0.0;
        for (int l = 0; l < k; ++l) s += (tx ? X[l * r + i] : X[i * k + l]) * v[l];
        y[i] = s;
    }
}

static void symmetrize(int n, double* S) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            double a = 0.5 * (S[i * n + j] + S[j * n + i]);
            S[i * n + j] = a;
            S[j * n + i] = a;
        }
}

/* Textbook Cholesky S = L L' (L lower, stored in place of the lower part).
 * Returns 0 on success, -1 if a pivot is not strictly positive. */
static int cholesky(int n, double* S) {
    for (int j = 0; j < n; ++j) {
        double d = S[j * n + j];
        for (int k = 0; k < j; ++k) d -= S[j * n + k] * S[j * n + k];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        S[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = S[i * n + j];
            for (int k = 0; k < j; ++k) s -= S[i * n + k] * S[j * n + k];
            S[i * n + j] = s / d;
        }
        for (int i = 0; i < j; ++i) S[i * n + j] = 0.0;
    }
    return 0;
}

/* Solve (L L') X = Y in place for nrhs right-hand sides stored as the
 * columns of the n x nrhs row-major matrix Y. */
static void chol_solve(int n, const double* L, int nrhs, double* Y) {
    for (int c = 0; c < nrhs; ++c) {
        for (int i = 0; i < n; ++i) {
            double s = Y[i * nrhs + c];
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * Y[k * nrhs + c];
            Y[i * nrhs + c] = s / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = Y[i * nrhs + c];
            for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * Y[k * nrhs + c];
            Y[i * nrhs + c] = s / L[i * n + i];
        }
    }
}

/* Solve E X = Y (E general n x n, Y n x nrhs, both row-major) by Gaussian
 * elimination with partial pivoting.  E and Y are overwritten.
 * Returns 0, or -1 on an exactly singular pivot. */
static int lu_solve(int n, double* E, int nrhs, double* Y) {
    for (int j = 0; j < n; ++j) {
        int piv = j;
        double best = fabs(E[j * n + j]);
        for (int i = j + 1; i < n; ++i)
            if (fabs(E[i * n + j]) > best) { best = fabs(E[i * n + j]); piv = i; }
        if (best == 0.0) return -1;
        if (piv != j) {
            for (int k = 0; k < n; ++k) { double t = E[j*n+k]; E[j*n+k] = E[piv*n+k]; E[piv*n+k] = t; }
            for (int k = 0; k < nrhs; ++k) { double t = Y[j*nrhs+k]; Y[j*nrhs+k] = Y[piv*nrhs+k]; Y[piv*nrhs+k] = t; }
        }
        for (int i = j + 1; i < n; ++i) {
            double f = E[i * n + j] / E[j * n + j];
            if (f == 0.0) continue;
            for (int k = j; k < n; ++k) E[i * n + k] -= f * E[j * n + k];
            for (int k = 0; k < nrhs; ++k) Y[i * nrhs + k] -= f * Y[j * nrhs + k];
        }
    }
    for (int i = n - 1; i >= 0; --i)
        for (int k = 0; k < nrhs; ++k) {
            double s = Y[i * nrhs + k];
            for (int l = i + 1; l < n; ++l) s -= E[i * n + l] * Y[l * nrhs + k];
            Y[i * nrhs + k] = s / E[i * n + i];
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Sec. II-C: Riccati recursion, forward pass, costates               */
/* ------------------------------------------------------------------ */

/*
 * Backward pass, eq. (lqr), with S_k = M_k':
 *   G = R + B'P'B,  H = S + B'P'A,  h = B'(p' + P'c) + r,
 *   K = -G^{-1}H,   k = -G^{-1}h,
 *   P = Q + A'P'A + K'H,  p = q + A'(p' + P'c) + K'h,
 * starting from P_N = Q_N, p_N = q_N (primes denote stage k+1).  P_k is
 * symmetrized after every step (round-off hygiene only).
 * Forward pass: u_k = K_k x_k + k_k, x_{k+1} = A_k x_k + B_k u_k + c_k.
 * Costates: lambda_k = P_k x_k + p_k.
 *
 * Optional outputs (may be NULL): P[N+1][n][n], p[N+1][n], K[N][m][n],
 * kff[N][m].  Returns 0, -1 on bad sizes / allocation, -2 if some G_k is not
 * positive definite.
 */
int lqro_riccati(int N, int n, int m, const double* A, const double* B,
                 const double* c, const double* Q, const double* R,
                 const double* M, const double* q, const double* r,
                 const double* x0, double* x, double* u, double* lam,
                 double* P_out, double* p_out, double* K_out, double* k_out) {
    if (N < 1 || n < 1 || m < 1) return -1;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m, mm_ = (size_t)m * m;
    double* P = (double*)malloc(sizeof(double) * (N + 1) * nn);
    double* p = (double*)malloc(sizeof(double) * (N + 1) * n);
    double* K = (double*)malloc(sizeof(double) * N * nm);
    double* kf = (double*)malloc(sizeof(double) * N * m);
    double* PA = (double*)malloc(sizeof(double) * nn);
    double* PB = (double*)malloc(sizeof(double) * nm);
    double* G = (double*)malloc(sizeof(double) * mm_);
    double* H = (double*)malloc(sizeof(double) * nm);
    double* T = (double*)malloc(sizeof(double) * nn);
    double* v = (double*)malloc(sizeof(double) * n);
    double* h = (double*)malloc(sizeof(double) * m);
    double* w = (double*)malloc(sizeof(double) * n);
    int rc = 0;
    if (!P || !p || !K || !kf || !PA || !PB || !G || !H || !T || !v || !h || !w) { rc = -1; goto done; }

    memcpy(P + (size_t)N * nn, Q + (size_t)N * nn, sizeof(double) * nn);
    memcpy(p + (size_t)N * n, q + (size_t)N * n, sizeof(double) * n);
    for (int k = N - 1; k >= 0; --k) {
        const double* Ak = A + k * nn; const double* Bk = B + k * nm;
        const double* ck = c + (size_t)k * n; const double* Qk = Q + k * nn;
        const double* Rk = R + k * mm_; const double* Mk = M + k * nm;
        const double* Pn = P + (size_t)(k + 1) * nn; const double* pn = p + (size_t)(k + 1) * n;
        mm(n, n, n, Pn, 0, Ak, 0, PA);           /* P' A           */
        mm(n, m, n, Pn, 0, Bk, 0, PB);           /* P' B           */
        mm(m, m, n, Bk, 1, PB, 0, G);            /* B' P' B        */
        for (size_t i = 0; i < mm_; ++i) G[i] += Rk[i];
        mm(m, n, n, Bk, 1, PA, 0, H);            /* B' P' A        */
        for (int i = 0; i < m; ++i)              /* + S = M'       */
            for (int j = 0; j < n; ++j) H[i * n + j] += Mk[j * m + i];
        mv(n, n, Pn, 0, ck, v);                  /* v = p' + P' c  */
        for (int i = 0; i < n; ++i) v[i] += pn[i];
        mv(m, n, Bk, 1, v, h);                   /* h = B' v + r   */
        for (int i = 0; i < m; ++i) h[i] += r[(size_t)k * m + i];
        symmetrize(m, G);
        if (cholesky(m, G) != 0) { rc = -2; goto done; }
        double* Kk = K + k * nm; double* kk = kf + (size_t)k * m;
        for (size_t i = 0; i < nm; ++i) Kk[i] = -H[i];
        chol_solve(m, G, n, Kk);                 /* K = -G^{-1} H  */
        for (int i = 0; i < m; ++i) kk[i] = -h[i];
        chol_solve(m, G, 1, kk);                 /* k = -G^{-1} h  */
        double* Pk = P + (size_t)k * nn; double* pk = p + (size_t)k * n;
        mm(n, n, n, Ak, 1, PA, 0, Pk);           /* A' P' A        */
        mm(n, n, m, Kk, 1, H, 0, T);             /* K' H           */
        for (size_t i = 0; i < nn; ++i) Pk[i] += Qk[i] + T[i];
        symmetrize(n, Pk);
        mv(n, n, Ak, 1, v, pk);                  /* A' v           */
        mv(n, m, Kk, 1, h, w);                   /* K' h           */
        for (int i = 0; i < n; ++i) pk[i] += q[(size_t)k * n + i] + w[i];
    }
    /* forward pass */
    memcpy(x, x0, sizeof(double) * n);
    for (int k = 0; k < N; ++k) {
        const double* xk = x + (size_t)k * n; double* uk = u + (size_t)k * m;
        double* xn = x + (size_t)(k + 1) * n;
        mv(m, n, K + k * nm, 0, xk, uk);
        for (int i = 0; i < m; ++i) uk[i] += kf[(size_t)k * m + i];
        mv(n, n, A + k * nn, 0, xk, xn);
        mv(n, m, B + k * nm, 0, uk, w);
        for (int i = 0; i < n; ++i) xn[i] += w[i] + c[(size_t)k * n + i];
    }
    /* costates */
    for (int k = 0; k <= N; ++k) {
        mv(n, n, P + (size_t)k * nn, 0, x + (size_t)k * n, lam + (size_t)k * n);
        for (int i = 0; i < n; ++i) lam[(size_t)k * n + i] += p[(size_t)k * n + i];
    }
    if (P_out) memcpy(P_out, P, sizeof(double) * (N + 1) * nn);
    if (p_out) memcpy(p_out, p, sizeof(double) * (N + 1) * n);
    if (K_out) memcpy(K_out, K, sizeof(double) * N * nm);
    if (k_out) memcpy(k_out, kf, sizeof(double) * N * m);
done:
    free(P); free(p); free(K); free(kf); free(PA); free(PB); free(G); free(H);
    free(T); free(v); free(h); free(w);
    return rc;
}

/* ------------------------------------------------------------------ */
/* batch driver: independent instances over a pthread pool             */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t batch; int N, n, m;
    const double *A, *B, *c, *Q, *R, *M, *q, *r, *x0;
    double *x, *u, *lam;
    int32_t* status;
    int64_t next;   /* work counter (atomic) */
} batch_job;

static void* batch_worker(void* arg) {
    batch_job* j = (batch_job*)arg;
    const size_t nn = (size_t)j->n * j->n, nm = (size_t)j->n * j->m, mm_ = (size_t)j->m * j->m;
    const size_t N = (size_t)j->N, n = (size_t)j->n, m = (size_t)j->m;
    for (;;) {
        int64_t b = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
        if (b >= j->batch) break;
        int rc = lqro_riccati(j->N, j->n, j->m, j->A + b * N * nn, j->B + b * N * nm,
                              j->c + b * N * n, j->Q + b * (N + 1) * nn, j->R + b * N * mm_,
                              j->M + b * N * nm, j->q + b * (N + 1) * n, j->r + b * N * m,
                              j->x0 + b * n, j->x + b * (N + 1) * n, j->u + b * N * m,
                              j->lam + b * (N + 1) * n, NULL, NULL, NULL, NULL);
        if (j->status) j->status[b] = rc;
    }
    return NULL;
}

/* Solves `batch` independent instances laid out batch-major (each array is
 * the single-instance layout repeated).  nthreads <= 0 means 1.  Returns the
 * number of instances whose solve failed. */
int64_t lqro_riccati_batch(int64_t batch, int N, int n, int m, const double* A,
                           const double* B, const double* c, const double* Q,
                           const double* R, const double* M, const double* q,
                           const double* r, const double* x0, double* x,
                           double* u, double* lam, int32_t* status,
                           int nthreads) {
    batch_job j = {batch, N, n, m, A, B, c, Q, R, M, q, r, x0, x, u, lam, status, 0};
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 512) nthreads = 512;
    pthread_t th[512];
    int started = 0;
    for (int t = 1; t < nthreads; ++t)
        if (pthread_create(&th[started], NULL, batch_worker, &j) == 0) ++started;
    batch_worker(&j);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    int64_t bad = 0;
    if (status)
        for (int64_t b = 0; b < batch; ++b) bad += status[b] != 0;
    return bad;
}

/* ------------------------------------------------------------------ */
/* Sec. II-B: KKT residual of the equality-constrained QP              */
/* ------------------------------------------------------------------ */

/*
 * Stationarity of the Lagrangian
 *   l_N(x_N) + lam_0'(x0 - x_0) + sum_k l_k(x_k,u_k) + lam_{k+1}'(A_k x_k + B_k u_k + c_k - x_{k+1})
 * plus primal feasibility.  The residual vector is stacked as
 *   [ r_init (n) | r_dyn[1..N] (N n) | r_x[0..N] ((N+1) n) | r_u[0..N-1] (N m) ]
 *   r_init   = x_0 - x0
 *   r_dyn    = A_k x_k + B_k u_k + c_k - x_{k+1}
 *   r_x[k]   = Q_k x_k + M_k u_k + q_k + A_k' lam_{k+1} - lam_k   (k < N)
 *   r_x[N]   = Q_N x_N + q_N - lam_N
 *   r_u[k]   = M_k' x_k + R_k u_k + r_k + B_k' lam_{k+1}
 * res may be NULL.  norms[0] = ||residual||_2, norms[1] = ||(x0, c, q, r)||_2.
 */
void lqro_kkt_residual(int N, int n, int m, const double* A, const double* B,
                       const double* c, const double* Q, const double* R,
                       const double* M, const double* q, const double* r,
                       const double* x0, const double* x, const double* u,
                       const double* lam, double* res, double* norms) {
    const size_t nn = (size_t)n * n, nm = (size_t)n * m, mm_ = (size_t)m * m;
    double* t1 = (double*)malloc(sizeof(double) * (n > m ? n : m));
    double* t2 = (double*)malloc(sizeof(double) * (n > m ? n : m));
    double rr = 0.0, bb = 0.0;
    size_t o = 0;
    for (int i = 0; i < n; ++i) {
        double e = x[i] - x0[i];
        if (res) res[o] = e;
        ++o; rr += e * e; bb += x0[i] * x0[i];
    }
    for (int k = 0; k < N; ++k) {
        mv(n, n, A + k * nn, 0, x + (size_t)k * n, t1);
        mv(n, m, B + k * nm, 0, u + (size_t)k * m, t2);
        for (int i = 0; i < n; ++i) {
            double ck = c[(size_t)k * n + i];
            double e = t1[i] + t2[i] + ck - x[(size_t)(k + 1) * n + i];
            if (res) res[o] = e;
            ++o; rr += e * e; bb += ck * ck;
        }
    }
    for (int k = 0; k <= N; ++k) {
        mv(n, n, Q + k * nn, 0, x + (size_t)k * n, t1);
        for (int i = 0; i < n; ++i) {
            double e = t1[i] + q[(size_t)k * n + i] - lam[(size_t)k * n + i];
            if (k < N) {
                double s = 0.0;
                for (int j = 0; j < m; ++j) s += M[k * nm + (size_t)i * m + j] * u[(size_t)k * m + j];
                for (int j = 0; j < n; ++j) s += A[k * nn + (size_t)j * n + i] * lam[(size_t)(k + 1) * n + j];
                e += s;
            }
            if (res) res[o] = e;
            ++o; rr += e * e; bb += q[(size_t)k * n + i] * q[(size_t)k * n + i];
        }
    }
    for (int k = 0; k < N; ++k) {
        mv(m, n, M + k * nm, 1, x + (size_t)k * n, t1);
        mv(m, m, R + k * mm_, 0, u + (size_t)k * m, t2);
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += B[k * nm + (size_t)j * m + i] * lam[(size_t)(k + 1) * n + j];
            double rk = r[(size_t)k * m + i];
            double e = t1[i] + t2[i] + rk + s;
            if (res) res[o] = e;
            ++o; rr += e * e; bb += rk * rk;
        }
    }
    norms[0] = sqrt(rr);
    norms[1] = sqrt(bb);
    free(t1); free(t2);
}

/* ------------------------------------------------------------------ */
/* Sec. II-D: conditional value functions and their combination        */
/* ------------------------------------------------------------------ */

/*
 * eq. (initialization): the one-stage conditional value function
 * V_{k->k+1}(x_k, x_{k+1}) in the dual form of eq. (conditional_value_function),
 * with S = M':
 *   At = A - B R^{-1} S,    Pt = Q - S' R^{-1} S,   Ct = B R^{-1} B',
 *   pt = q - S' R^{-1} r,   bt = c - B R^{-1} r.
 * (The constant -1/2 r'R^{-1}r of the stage is dropped, as in the paper; it
 * does not influence x, u or lambda.)  Pt and Ct are symmetrized.
 * The terminal element is (At, bt, Ct, Pt, pt) = (0, 0, 0, Q_N, q_N) and is
 * formed by the caller.  Returns 0, or -2 if R is not positive definite.
 */
int lqro_element(int n, int m, const double* A, const double* B,
                 const double* c, const double* Q, const double* R,
                 const double* M, const double* q, const double* r,
                 double* At, double* bt, double* Ct, double* Pt, double* pt) {
    const int w = 2 * n + 1;   /* columns of the right-hand side [M' | B' | r] */
    double* L = (double*)malloc(sizeof(double) * m * m);
    double* Y = (double*)malloc(sizeof(double) * m * w);
    memcpy(L, R, sizeof(double) * m * m);
    symmetrize(m, L);
    int rc = cholesky(m, L);
    if (rc != 0) { rc = -2; goto done; }
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) {
            Y[i * w + j] = M[j * m + i];          /* S  = M'  */
            Y[i * w + n + j] = B[j * m + i];      /* B'       */
        }
        Y[i * w + 2 * n] = r[i];
    }
    chol_solve(m, L, w, Y);                       /* Y = R^{-1}[S | B' | r] */
    /* split views of Y: RS = R^{-1}S (m x n), RB = R^{-1}B' (m x n), Rr (m) */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double bs = 0.0, ss = 0.0, bb = 0.0;
            for (int l = 0; l < m; ++l) {
                bs += B[i * m + l] * Y[l * w + j];        /* B R^{-1} S   */
                ss += M[i * m + l] * Y[l * w + j];        /* S' R^{-1} S  */
                bb += B[i * m + l] * Y[l * w + n + j];    /* B R^{-1} B'  */
            }
            At[i * n + j] = A[i * n + j] - bs;
            Pt[i * n + j] = Q[i * n + j] - ss;
            Ct[i * n + j] = bb;
        }
    for (int i = 0; i < n; ++i) {
        double sr = 0.0, br = 0.0;
        for (int l = 0; l < m; ++l) {
            sr += M[i * m + l] * Y[l * w + 2 * n];
            br += B[i * m + l] * Y[l * w + 2 * n];
        }
        pt[i] = q[i] - sr;
        bt[i] = c[i] - br;
    }
    symmetrize(n, Pt);
    symmetrize(n, Ct);
done:
    free(L); free(Y);
    return rc;
}

/*
 * eq. (combination_rule): V_{i->j} = min_{x_k} V_{i->k} + V_{k->j}, with
 * element 1 = (A1,b1,C1,P1,p1) for the earlier segment i->k and element 2 for
 * the later segment k->j.  Writing E = I + C1 P2:
 *   A = A2 E^{-1} A1
 *   C = A2 E^{-1} C1 A2' + C2
 *   b = A2 E^{-1} (b1 - C1 p2) + b2
 *   P = A1' E^{-T} P2 A1 + P1             (E^{-T} = (I + P2 C1)^{-1})
 *   p = A1' E^{-T} (p2 + P2 b1) + p1
 * The A, C and P rules are as printed.  The printed p and b rules carry index
 * and sign slips; the forms above are the ones obtained by minimizing the sum
 * of the two dual-form quadratics over x_k (and the only ones that reproduce
 * the Riccati value function of Sec. II-C).  Outputs may not alias inputs.
 * Returns 0, or -2 if E is singular.
 */
int lqro_combine(int n, const double* A1, const double* b1, const double* C1,
                 const double* P1, const double* p1, const double* A2,
                 const double* b2, const double* C2, const double* P2,
                 const double* p2, double* A, double* b, double* C, double* P,
                 double* p) {
    const size_t nn = (size_t)n * n;
    const int w = 2 * n + 1;
    double* E = (double*)malloc(sizeof(double) * nn);
    double* Y = (double*)malloc(sizeof(double) * n * w);
    double* T = (double*)malloc(sizeof(double) * nn);
    double* t = (double*)malloc(sizeof(double) * n);
    int rc = 0;
    /* E = I + C1 P2;  solve E Y = [A1 | C1 | b1 - C1 p2] */
    mm(n, n, n, C1, 0, P2, 0, E);
    for (int i = 0; i < n; ++i) E[i * n + i] += 1.0;
    mv(n, n, C1, 0, p2, t);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            Y[i * w + j] = A1[i * n + j];
            Y[i * w + n + j] = C1[i * n + j];
        }
        Y[i * w + 2 * n] = b1[i] - t[i];
    }
    if (lu_solve(n, E, w, Y) != 0) { rc = -2; goto done; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double sa = 0.0, sc = 0.0;
            for (int l = 0; l < n; ++l) {
                sa += A2[i * n + l] * Y[l * w + j];
                sc += A2[i * n + l] * Y[l * w + n + j];
            }
            A[i * n + j] = sa;
            T[i * n + j] = sc;                   /* A2 E^{-1} C1 */
        }
    mm(n, n, n, T, 0, A2, 1, C);                 /* (A2 E^{-1} C1) A2' */
    for (size_t i = 0; i < nn; ++i) C[i] += C2[i];
    symmetrize(n, C);
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int l = 0; l < n; ++l) s += A2[i * n + l] * Y[l * w + 2 * n];
        b[i] = s + b2[i];
    }
    /* E' = I + P2 C1;  solve E' Z = [P2 A1 | p2 + P2 b1] */
    {
        const int w2 = n + 1;
        double* Z = (double*)malloc(sizeof(double) * n * w2);
        mm(n, n, n, P2, 0, C1, 0, E);
        for (int i = 0; i < n; ++i) E[i * n + i] += 1.0;
        mm(n, n, n, P2, 0, A1, 0, T);
        mv(n, n, P2, 0, b1, t);
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) Z[i * w2 + j] = T[i * n + j];
            Z[i * w2 + n] = p2[i] + t[i];
        }
        if (lu_solve(n, E, w2, Z) != 0) { free(Z); rc = -2; goto done; }
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int l = 0; l < n; ++l) s += A1[l * n + i] * Z[l * w2 + j];
                P[i * n + j] = s + P1[i * n + j];
            }
            double s = 0.0;
            for (int l = 0; l < n; ++l) s += A1[l * n + i] * Z[l * w2 + n];
            p[i] = s + p1[i];
        }
        symmetrize(n, P);
        free(Z);
    }
done:
    free(E); free(Y); free(T); free(t);
    return rc;
}

/*
 * Composition of conditional optimal trajectories dx_j = Abar dx_i + bbar
 * (eq. controlled_dynamics / conditional_optimal_trajectory): applying the
 * earlier map (M1, v1) first and the later map (M2, v2) second gives
 *   M = M2 M1,   v = M2 v1 + v2.
 * The printed product has the factors in the other order, which does not
 * compose the two maps; the b-part is as printed.  Outputs may not alias.
 */
void lqro_affine_combine(int n, const double* M1, const double* v1,
                         const double* M2, const double* v2, double* M,
                         double* v) {
    mm(n, n, n, M2, 0, M1, 0, M);
    mv(n, n, M2, 0, v1, v);
    for (int i = 0; i < n; ++i) v[i] += v2[i];
}
