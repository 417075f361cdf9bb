// qpdata.hpp -- the QP-data builder that precedes the KKT solve (gfx950).
//
// Paper: Amatucci, Sousa-Pinto et al., arXiv 2506.07823, Sec. II-F.  The
// stage cost is a nonlinear least-squares term 1/2 eps' W eps plus relaxed
// barriers B(xi_j) of inequality constraints xi_j(x, u) >= 0.  With the
// Gauss-Newton approximation (second derivatives of eps and xi dropped)
// the blocks of stage k, in the ABI's convention (M = S', n x m), are
//   Q = Ex' W Ex + Gx' D2 Gx,  M = Ex' W Eu + Gx' D2 Gu,  R = Eu' W Eu + Gu' D2 Gu,
//   q = Ex' W eps + Gx' D1,    r = Eu' W eps + Gu' D1,
// D1 = B'(xi), D2 = diag(B''(xi)) of the relaxed barrier
//   B = -mu ln(xi) for xi >= delta,  mu/2 (((xi - 2 delta)/delta)^2 - 1) - mu ln(delta) below,
// (mu, delta per constraint).  The terminal stage has no control part.
//
// One 256-thread workgroup per (instance, stage): W J (J = [Ex | Eu], p x d)
// is formed in LDS once, then every thread computes entries of J' (W J) +
// G' D2 G (lower triangle, mirrored) and of the gradient.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lqr {

template <typename S>
struct QpArgs {
    int64_t batch;
    int N, n, m, p, nc;
    const S *Ex, *Eu, *e, *W, *Gx, *Gu, *g, *mu, *delta;
    S *Q, *M, *R, *q, *r;
};

// first and second derivative of the relaxed barrier at xi
template <typename T>
__device__ __forceinline__ void barrier_d12(T xi, T mu, T delta, T& d1, T& d2) {
    if (xi >= delta) {
        d1 = -mu / xi;
        d2 = mu / (xi * xi);
    } else {
        d1 = mu * (xi - T(2) * delta) / (delta * delta);
        d2 = mu / (delta * delta);
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_qp_build(QpArgs<S> a) {
    extern __shared__ __align__(16) unsigned char qp_lds[];
    const int N = a.N, n = a.n, m = a.m, p = a.p, nc = a.nc;
    const int64_t b = blockIdx.x / (N + 1);
    const int k = (int)(blockIdx.x % (N + 1));
    const bool term = k == N;
    const int d = term ? n : n + m;
    const int64_t sx = b * (N + 1) + k;   // stage index of the x-side arrays
    const int64_t su = b * N + k;         // of the u-side arrays
    const S* Ex = a.Ex + sx * p * n;
    const S* Eu = term ? nullptr : a.Eu + su * p * m;
    const S* e = a.e + sx * p;
    const S* W = a.W + sx * p * p;
    const S* Gx = nc ? a.Gx + sx * nc * n : nullptr;
    const S* Gu = (nc && !term) ? a.Gu + su * nc * m : nullptr;
    const S* g = nc ? a.g + sx * nc : nullptr;
    S* WJ = reinterpret_cast<S*>(qp_lds);   // [p][d]
    S* We = WJ + p * d;                     // [p]
    S* D1 = We + p;                         // [nc]
    S* D2 = D1 + nc;                        // [nc]
    auto J = [&](int row, int j) -> S { return j < n ? Ex[row * n + j] : Eu[row * m + (j - n)]; };
    auto G = [&](int row, int j) -> S { return j < n ? Gx[row * n + j] : Gu[row * m + (j - n)]; };
    const int t = threadIdx.x;
    for (int idx = t; idx < p * d; idx += blockDim.x) {
        const int row = idx / d, j = idx - row * d;
        S s = S(0);
        for (int c = 0; c < p; ++c) s += W[row * p + c] * J(c, j);
        WJ[idx] = s;
    }
    for (int row = t; row < p; row += blockDim.x) {
        S s = S(0);
        for (int c = 0; c < p; ++c) s += W[row * p + c] * e[c];
        We[row] = s;
    }
    for (int c = t; c < nc; c += blockDim.x) barrier_d12<S>(g[c], a.mu[c], a.delta[c], D1[c], D2[c]);
    __syncthreads();
    // Hessian blocks: entry (i, j), i >= j, of [[Q, M], [M', R]]
    for (int idx = t; idx < d * d; idx += blockDim.x) {
        const int i = idx / d, j = idx - i * d;
        if (j > i) continue;
        S h = S(0);
        for (int c = 0; c < p; ++c) h += J(c, i) * WJ[c * d + j];
        for (int c = 0; c < nc; ++c) h += G(c, i) * D2[c] * G(c, j);
        if (i < n) {
            S* Q = a.Q + sx * n * n;
            Q[i * n + j] = h;
            Q[j * n + i] = h;
        } else if (j < n) {
            a.M[su * n * m + j * m + (i - n)] = h;
        } else {
            S* R = a.R + su * m * m;
            R[(i - n) * m + (j - n)] = h;
            R[(j - n) * m + (i - n)] = h;
        }
    }
    // gradient
    for (int i = t; i < d; i += blockDim.x) {
        S v = S(0);
        for (int c = 0; c < p; ++c) v += J(c, i) * We[c];
        for (int c = 0; c < nc; ++c) v += G(c, i) * D1[c];
        if (i < n) a.q[sx * n + i] = v;
        else a.r[su * m + (i - n)] = v;
    }
}

}  // namespace lqr
