"""CPU FP64 oracle of the QP-data builder (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this module; the GPU product path never imports, links or
calls it, and the two share no code.  Plain numpy, FP64, one stage at a
time.

Paper: Amatucci, Sousa-Pinto et al., arXiv 2506.07823, Sec. II-F (Practical
Implementation).  The stage cost is a nonlinear least-squares term
1/2 eps' W eps plus relaxed barriers B(xi_j) of the inequality constraints
xi_j(x, u) >= 0.  With the Gauss-Newton approximation (second derivatives
of eps and xi dropped) the QP blocks of a stage are

    Q = Ex' W Ex + Gx' diag(B''(xi)) Gx        (n x n)
    S' = M = Ex' W Eu + Gx' diag(B''(xi)) Gu   (n x m, the ABI's cross term)
    R = Eu' W Eu + Gu' diag(B''(xi)) Gu        (m x m)

and the linear terms are the cost gradient

    q = Ex' W eps + Gx' B'(xi),   r = Eu' W eps + Gu' B'(xi),

with Ex, Eu the Jacobians of eps and Gx, Gu those of xi.  The terminal stage
has no control part.  The relaxed barrier of one constraint, with its
parameters mu > 0 and delta > 0, is

    B(xi) = -mu ln(xi)                                           xi >= delta
    B(xi) = mu/2 (((xi - 2 delta) / delta)^2 - 1) - mu ln(delta)  xi < delta

Readings (the paper is garbled or silent here): the constraint is feasible
for xi >= 0 (the log branch needs xi > 0); the printed S block of the
barrier form repeats the x-x product, read as Ex' W Eu like the plain
Gauss-Newton form; the linear terms, which the paper does not print, are
the gradient of the same cost.
"""
from __future__ import annotations

import numpy as np


def barrier(xi, mu, delta):
    """Relaxed barrier value (Sec. II-F), elementwise."""
    xi, mu, delta = np.broadcast_arrays(np.asarray(xi, float), np.asarray(mu, float), np.asarray(delta, float))
    out = np.empty_like(xi)
    hi = xi >= delta
    out[hi] = -mu[hi] * np.log(xi[hi])
    lo = ~hi
    out[lo] = mu[lo] / 2 * (((xi[lo] - 2 * delta[lo]) / delta[lo]) ** 2 - 1) - mu[lo] * np.log(delta[lo])
    return out


def barrier_d1(xi, mu, delta):
    """dB/dxi: -mu/xi on the log branch, mu (xi - 2 delta) / delta^2 below delta."""
    xi, mu, delta = np.broadcast_arrays(np.asarray(xi, float), np.asarray(mu, float), np.asarray(delta, float))
    return np.where(xi >= delta, -mu / np.where(xi >= delta, xi, 1.0), mu * (xi - 2 * delta) / delta ** 2)


def barrier_d2(xi, mu, delta):
    """d2B/dxi2: mu/xi^2 on the log branch, mu/delta^2 below delta."""
    xi, mu, delta = np.broadcast_arrays(np.asarray(xi, float), np.asarray(mu, float), np.asarray(delta, float))
    return np.where(xi >= delta, mu / np.where(xi >= delta, xi, 1.0) ** 2, mu / delta ** 2)


def build_stage(Ex, e, W, Gx, g, mu, delta, Eu=None, Gu=None):
    """QP blocks of one stage (Sec. II-F); Eu, Gu None for the terminal
    stage.  Returns (Q, M, R, q, r) with M, R, r None at the terminal stage."""
    Ex, e, W = np.asarray(Ex, float), np.asarray(e, float), np.asarray(W, float)
    Gx, g = np.asarray(Gx, float).reshape(-1, Ex.shape[1]), np.asarray(g, float).reshape(-1)
    d2 = barrier_d2(g, mu, delta)
    d1 = barrier_d1(g, mu, delta)
    We = W @ e
    Q = Ex.T @ W @ Ex + Gx.T @ (d2[:, None] * Gx)
    q = Ex.T @ We + Gx.T @ d1
    if Eu is None:
        return Q, None, None, q, None
    Eu, Gu = np.asarray(Eu, float), np.asarray(Gu, float).reshape(-1, Eu.shape[1])
    M = Ex.T @ W @ Eu + Gx.T @ (d2[:, None] * Gu)
    R = Eu.T @ W @ Eu + Gu.T @ (d2[:, None] * Gu)
    r = Eu.T @ We + Gu.T @ d1
    return Q, M, R, q, r


def build(d):
    """Every stage of every instance of a batch dict (synth.gen_qpdata
    layout); returns Q, M, R, q, r with a leading batch axis."""
    Ex, Eu, e, W = d["Ex"], d["Eu"], d["e"], d["W"]
    Gx, Gu, g, mu, delta = d["Gx"], d["Gu"], d["g"], d["mu"], d["delta"]
    B, N1, p, n = Ex.shape
    N, m = N1 - 1, Eu.shape[-1]
    out = {"Q": np.zeros((B, N + 1, n, n)), "M": np.zeros((B, N, n, m)), "R": np.zeros((B, N, m, m)),
           "q": np.zeros((B, N + 1, n)), "r": np.zeros((B, N, m))}
    for b in range(B):
        for k in range(N + 1):
            if k < N:
                Q, M, R, q, r = build_stage(Ex[b, k], e[b, k], W[b, k], Gx[b, k], g[b, k], mu, delta,
                                            Eu[b, k], Gu[b, k])
                out["M"][b, k], out["R"][b, k], out["r"][b, k] = M, R, r
            else:
                Q, _, _, q, _ = build_stage(Ex[b, k], e[b, k], W[b, k], Gx[b, k], g[b, k], mu, delta)
            out["Q"][b, k], out["q"][b, k] = Q, q
    return out
