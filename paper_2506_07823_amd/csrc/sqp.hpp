// sqp.hpp -- the SQP iteration around the KKT solve on a synthetic nonlinear
// model (gfx950): linearization, parallel filter line search, update.
//
// Paper: Amatucci, Sousa-Pinto et al., arXiv 2506.07823, Sec. II-B (the
// subproblem of one SQP iteration), II-E (parallel line search), II-F
// (Gauss-Newton blocks, relaxed barriers).  Model (a stand-in for the robot
// models): dynamics with a bilinear term, h(x, u) = A x + B u + c +
// gamma (P x) * (V u) (elementwise product), a tracking cost with diagonal
// weights, linear inequality constraints xi = Gx x + Gu u + g0 >= 0 under the
// relaxed barrier.  Every kernel runs one 64-lane workgroup per task; lane i
// owns row i (orders up to 64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qpdata.hpp"

namespace lqr {

constexpr int kAlphas = 10;   // trial steps 2^0 .. 2^-9

template <typename S>
struct SqpModel {
    int64_t batch;
    int N, n, m, nc;
    const S *A, *B, *c, *P, *V;          // [b][n][n], [b][n][m], [b][n], [b][n][n], [b][n][m]
    const S *xr, *ur, *wx, *wu;          // [b][N+1][n], [b][N][m], [b][N+1][n], [b][N][m]
    const S *Gx, *Gu, *g0, *mu, *delta;  // [b][nc][n], [b][nc][m], [b][nc], [nc], [nc]
    const S* xhat0;                      // [b][n]
    double gamma;
};

// the subproblem's arrays and the line search's per-trial sums
template <typename S>
struct SqpWork {
    S *A, *B, *c, *x0;                   // dynamics part of the subproblem (solve layout)
    S *Ex, *Eu, *e, *W, *Gx, *Gu, *g;    // QP-builder inputs (p = n + m rows)
    S *Q, *M, *R, *q, *r;                // QP-builder outputs
    S *dx, *du, *lqp;                    // the subproblem's solution
    double *th, *J, *dJ;                 // [b][kAlphas + 1] (trial 0: alpha = 0), [b]
};

__device__ __forceinline__ double wsum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// y_i = sum_j M_ij v_j for i < rows (lane i), M row-major with `cols` columns;
// v staged in LDS
template <typename T, typename S>
__device__ __forceinline__ T row_mv(const S* M, int rows, int cols, const T* v) {
    const int i = threadIdx.x;
    T s = T(0);
    if (i < rows)
        for (int j = 0; j < cols; ++j) s += T(M[(int64_t)i * cols + j]) * v[j];
    return s;
}

// relaxed barrier value (Sec. II-F)
__device__ __forceinline__ double barrier_value(double xi, double mu, double delta) {
    if (xi >= delta) return -mu * log(xi);
    const double t = (xi - 2.0 * delta) / delta;
    return 0.5 * mu * (t * t - 1.0) - mu * log(delta);
}

// Constant parts of the QP-builder inputs (once per solve): the selection
// Jacobians of the tracking residual, the weights and the constraint
// Jacobians, replicated per stage.  One workgroup per (instance, stage).
template <typename S>
__global__ __launch_bounds__(64) void k_sqp_setup(SqpModel<S> md, SqpWork<S> w) {
    const int N = md.N, n = md.n, m = md.m, nc = md.nc, p = n + m;
    const int64_t b = blockIdx.x / (N + 1);
    const int k = (int)(blockIdx.x % (N + 1));
    const int64_t sx = b * (N + 1) + k, su = b * N + k;
    for (int idx = threadIdx.x; idx < p * n; idx += 64) {
        const int r = idx / n, j = idx - r * n;
        w.Ex[sx * p * n + idx] = S(r == j ? 1 : 0);
    }
    for (int idx = threadIdx.x; idx < p * p; idx += 64) {
        const int r = idx / p, j = idx - r * p;
        S v = S(0);
        if (r == j) v = r < n ? md.wx[sx * n + r] : (k < N ? md.wu[su * m + (r - n)] : S(0));
        w.W[sx * p * p + idx] = v;
    }
    for (int idx = threadIdx.x; idx < nc * n; idx += 64) w.Gx[sx * nc * n + idx] = md.Gx[b * nc * n + idx];
    if (k < N) {
        for (int idx = threadIdx.x; idx < p * m; idx += 64) {
            const int r = idx / m, j = idx - r * m;
            w.Eu[su * p * m + idx] = S(r == n + j ? 1 : 0);
        }
        for (int idx = threadIdx.x; idx < nc * m; idx += 64) w.Gu[su * nc * m + idx] = md.Gu[b * nc * m + idx];
    }
}

// Linearization at the iterate (X, U) (Sec. II-B): A_k = dh/dx, B_k = dh/du,
// c_k = h(x_k, u_k) - x_{k+1} (so that the subproblem's dynamics are those
// of the step), the tracking residual e_k and constraint values g_k for the
// QP builder, and x0 = xhat0 - x_0.  One workgroup per (instance, stage).
template <typename S>
__global__ __launch_bounds__(64) void k_sqp_linearize(SqpModel<S> md, SqpWork<S> w, const S* X, const S* U) {
    __shared__ double xs[64], us[64];
    const int N = md.N, n = md.n, m = md.m, nc = md.nc, p = n + m;
    const int64_t b = blockIdx.x / (N + 1);
    const int k = (int)(blockIdx.x % (N + 1));
    const int i = threadIdx.x;
    const int64_t sx = b * (N + 1) + k, su = b * N + k;
    const S* x = X + sx * n;
    if (i < n) xs[i] = double(x[i]);
    if (k < N && i < m) us[i] = double(U[su * m + i]);
    __syncthreads();
    // residual and constraint values
    if (i < n) w.e[sx * p + i] = S(xs[i] - double(md.xr[sx * n + i]));
    if (i < m) w.e[sx * p + n + i] = k < N ? S(us[i] - double(md.ur[su * m + i])) : S(0);
    if (i < nc) {
        double v = double(md.g0[b * nc + i]);
        for (int j = 0; j < n; ++j) v += double(md.Gx[(b * nc + i) * n + j]) * xs[j];
        if (k < N)
            for (int j = 0; j < m; ++j) v += double(md.Gu[(b * nc + i) * m + j]) * us[j];
        w.g[sx * nc + i] = S(v);
    }
    if (k == 0 && i < n) w.x0[b * n + i] = S(double(md.xhat0[b * n + i]) - xs[i]);
    if (k == N) return;
    const S* A = md.A + b * n * n;
    const S* B = md.B + b * n * m;
    const S* P = md.P + b * n * n;
    const S* V = md.V + b * n * m;
    const double px = row_mv<double>(P, n, n, xs), vu = row_mv<double>(V, n, m, us);
    const double ax = row_mv<double>(A, n, n, xs), bu = row_mv<double>(B, n, m, us);
    const double g = md.gamma;
    if (i < n) {
        for (int j = 0; j < n; ++j)
            w.A[(su * n + i) * n + j] = S(double(A[i * n + j]) + g * vu * double(P[i * n + j]));
        for (int j = 0; j < m; ++j)
            w.B[(su * n + i) * m + j] = S(double(B[i * m + j]) + g * px * double(V[i * m + j]));
        const double h = ax + bu + double(md.c[b * n + i]) + g * px * vu;
        w.c[su * n + i] = S(h - double(X[(sx + 1) * n + i]));
    }
}

// Line search (Sec. II-E): trial t of instance b (t = 0: alpha = 0, else
// alpha = 2^-(t-1)): the dynamics violation theta = sum_k ||x_{k+1} -
// h(x_k, u_k)||_2 and the cost J at (X + alpha dX, U + alpha dU), FP64
// sums.  Trial 0 also forms the cost's directional derivative along the
// step from the subproblem's gradient, dJ = sum_k q_k'dx_k + r_k'du_k.
template <typename S>
__global__ __launch_bounds__(64) void k_sqp_trials(SqpModel<S> md, SqpWork<S> w, const S* X, const S* U) {
    __shared__ double xs[64], us[64];
    const int N = md.N, n = md.n, m = md.m, nc = md.nc;
    const int64_t b = blockIdx.x / (kAlphas + 1);
    const int t = (int)(blockIdx.x % (kAlphas + 1));
    const double alpha = t == 0 ? 0.0 : ldexp(1.0, -(t - 1));
    const int i = threadIdx.x;
    const S* A = md.A + b * n * n;
    const S* B = md.B + b * n * m;
    const S* P = md.P + b * n * n;
    const S* V = md.V + b * n * m;
    const double g = md.gamma;
    double th = 0.0, J = 0.0, dJ = 0.0;
    // iterate of stage k into LDS; returns lane i's state entry
    auto load = [&](int k) {
        const int64_t sx = b * (N + 1) + k, su = b * N + k;
        __syncthreads();
        if (i < n) xs[i] = double(X[sx * n + i]) + alpha * double(w.dx[sx * n + i]);
        if (k < N && i < m) us[i] = double(U[su * m + i]) + alpha * double(w.du[su * m + i]);
        __syncthreads();
    };
    for (int k = 0; k <= N; ++k) {
        const int64_t sx = b * (N + 1) + k, su = b * N + k;
        load(k);
        // stage cost
        double l = 0.0;
        if (i < n) {
            const double d = xs[i] - double(md.xr[sx * n + i]);
            l += 0.5 * double(md.wx[sx * n + i]) * d * d;
        }
        if (k < N && i < m) {
            const double d = us[i] - double(md.ur[su * m + i]);
            l += 0.5 * double(md.wu[su * m + i]) * d * d;
        }
        if (i < nc) {
            double v = double(md.g0[b * nc + i]);
            for (int j = 0; j < n; ++j) v += double(md.Gx[(b * nc + i) * n + j]) * xs[j];
            if (k < N)
                for (int j = 0; j < m; ++j) v += double(md.Gu[(b * nc + i) * m + j]) * us[j];
            l += barrier_value(v, double(md.mu[i]), double(md.delta[i]));
        }
        J += l;
        if (t == 0) {
            double dd = i < n ? double(w.q[sx * n + i]) * double(w.dx[sx * n + i]) : 0.0;
            if (k < N && i < m) dd += double(w.r[su * m + i]) * double(w.du[su * m + i]);
            dJ += dd;
        }
        if (k == N) break;
        // defect of the dynamics into stage k+1
        const double px = row_mv<double>(P, n, n, xs), vu = row_mv<double>(V, n, m, us);
        const double h = row_mv<double>(A, n, n, xs) + row_mv<double>(B, n, m, us) +
                         (i < n ? double(md.c[b * n + i]) + g * px * vu : 0.0);
        const double xn = i < n ? double(X[(sx + 1) * n + i]) + alpha * double(w.dx[(sx + 1) * n + i]) : 0.0;
        const double dfc = i < n ? xn - h : 0.0;
        th += __builtin_sqrt(wsum64(dfc * dfc));
    }
    J = wsum64(J);
    if (i == 0) {
        w.th[b * (kAlphas + 1) + t] = th;
        w.J[b * (kAlphas + 1) + t] = J;
    }
    if (t == 0) {
        dJ = wsum64(dJ);
        if (i == 0) w.dJ[b] = dJ;
    }
}

// Filter acceptance of one trial (Sec. II-E)
__device__ __forceinline__ bool filter_accepts(double th0, double J0, double th, double J, double alpha, double dJ,
                                               double theta_max, double eta) {
    if (th0 > theta_max) return th < th0;
    if (dJ < 0.0) return J <= J0 + eta * alpha * dJ;
    return J < J0 || th < th0;
}

// The largest accepted alpha (0 if none: status bit 32), and the update
//   X += alpha dX,  U += alpha dU,  L += alpha (lam_QP - L).
// One workgroup per instance.
template <typename S>
__global__ __launch_bounds__(64) void k_sqp_update(SqpModel<S> md, SqpWork<S> w, S* X, S* U, S* L, S* alpha_out,
                                                   int32_t* status, double theta_max, double eta) {
    __shared__ double sh_alpha;
    const int N = md.N, n = md.n, m = md.m;
    const int64_t b = blockIdx.x;
    if (threadIdx.x == 0) {
        const double* th = w.th + b * (kAlphas + 1);
        const double* J = w.J + b * (kAlphas + 1);
        double a = 0.0;
        for (int t = 1; t <= kAlphas; ++t) {
            const double at = ldexp(1.0, -(t - 1));
            if (filter_accepts(th[0], J[0], th[t], J[t], at, w.dJ[b], theta_max, eta)) {
                a = at;
                break;
            }
        }
        sh_alpha = a;
        if (alpha_out) alpha_out[b] = S(a);
        if (a == 0.0) atomicOr(status + b, 32);
    }
    __syncthreads();
    const double a = sh_alpha;
    if (a == 0.0) return;
    for (int64_t idx = threadIdx.x; idx < (int64_t)(N + 1) * n; idx += 64) {
        const int64_t o = b * (N + 1) * n + idx;
        X[o] = S(double(X[o]) + a * double(w.dx[o]));
        L[o] = S(double(L[o]) + a * (double(w.lqp[o]) - double(L[o])));
    }
    for (int64_t idx = threadIdx.x; idx < (int64_t)N * m; idx += 64) {
        const int64_t o = b * N * m + idx;
        U[o] = S(double(U[o]) + a * double(w.du[o]));
    }
}

}  // namespace lqr
