"""Independent brute-force constructions used to pin the oracle.

Nothing here reuses the oracle's recursions: the dense KKT matrix is built
from the QP statement itself (Sec. II-B, eq. (QP) and the Lagrangian), and
conditional value functions are evaluated by solving the segment's
equality-constrained QP densely with LAPACK (numpy.linalg).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def unknown_layout(N, n, m):
    """Offsets of x_0..x_N, u_0..u_{N-1}, lam_0..lam_N in the stacked vector."""
    nx = (N + 1) * n
    nu = N * m
    return nx, nu, nx + nu


def dense_kkt(prob):
    """Assemble [[H, E'], [E, 0]] and the right-hand side for the QP
        min sum_k 1/2 [x;u]'[[Q, M],[M', R]][x;u] + q'x + r'u + terminal
        s.t. x0 - x_0 = 0,  A_k x_k + B_k u_k + c_k - x_{k+1} = 0,
    with multipliers ordered lam_0 (initial condition), lam_{k+1} (dynamics
    of stage k), so that stationarity reads H z + g + E' lam = 0 and
    feasibility E z + e = 0.  Unknowns [x_0..x_N, u_0..u_{N-1}, lam_0..lam_N]."""
    A, B, c, Q, R, M, q, r, x0 = (prob[k] for k in ("A", "B", "c", "Q", "R", "M", "q", "r", "x0"))
    N, n, m = B.shape
    nx, nu, nz = unknown_layout(N, n, m)
    nl = (N + 1) * n
    H = np.zeros((nz, nz)); g = np.zeros(nz)
    xs = lambda k: slice(k * n, (k + 1) * n)
    us = lambda k: slice(nx + k * m, nx + (k + 1) * m)
    for k in range(N + 1):
        H[xs(k), xs(k)] += Q[k]
        g[xs(k)] += q[k]
    for k in range(N):
        H[us(k), us(k)] += R[k]
        H[xs(k), us(k)] += M[k]
        H[us(k), xs(k)] += M[k].T
        g[us(k)] += r[k]
    E = np.zeros((nl, nz)); e = np.zeros(nl)
    E[0:n, xs(0)] = -np.eye(n); e[0:n] = x0
    for k in range(N):
        rows = slice((k + 1) * n, (k + 2) * n)
        E[rows, xs(k)] += A[k]
        E[rows, us(k)] += B[k]
        E[rows, xs(k + 1)] += -np.eye(n)
        e[rows] = c[k]
    K = np.block([[H, E.T], [E, np.zeros((nl, nl))]])
    rhs = np.concatenate([-g, -e])
    return K, rhs


def dense_solve(prob):
    """Solve the dense KKT system; returns x [N+1][n], u [N][m], lam [N+1][n]."""
    N, n, m = prob["B"].shape
    K, rhs = dense_kkt(prob)
    z = np.linalg.solve(K, rhs)
    nx, nu, nz = unknown_layout(N, n, m)
    return z[:nx].reshape(N + 1, n), z[nx:nz].reshape(N, m), z[nz:].reshape(N + 1, n)


def stage_cost(Q, R, M, q, r, x, u):
    return 0.5 * x @ Q @ x + 0.5 * u @ R @ u + x @ M @ u + q @ x + r @ u


def qp_cost(prob, x, u):
    N = prob["B"].shape[0]
    J = sum(stage_cost(prob["Q"][k], prob["R"][k], prob["M"][k], prob["q"][k], prob["r"][k], x[k], u[k])
            for k in range(N))
    return J + 0.5 * x[N] @ prob["Q"][N] @ x[N] + prob["q"][N] @ x[N]


def segment_value(stages, xi, xj):
    """Brute force V_{i->j}(xi, xj): minimum total stage cost of the stages in
    ``stages`` (list of (A, B, c, Q, R, M, q, r)) over the controls and the
    intermediate states, with both end states fixed.  Returns None if the
    end state is unreachable (constraint inconsistent)."""
    L = len(stages)
    n, m = stages[0][1].shape
    nvar = L * m + (L - 1) * n          # u_i..u_{j-1}, x_{i+1}..x_{j-1}
    us = lambda k: slice(k * m, (k + 1) * m)
    xs = lambda k: slice(L * m + (k - 1) * n, L * m + k * n)   # k = 1..L-1
    H = np.zeros((nvar, nvar)); g = np.zeros(nvar); const = 0.0
    Ecs = np.zeros((L * n, nvar)); ecs = np.zeros(L * n)
    for k, (A, B, c, Q, R, M, q, r) in enumerate(stages):
        H[us(k), us(k)] += R
        g[us(k)] += r
        if k == 0:
            const += 0.5 * xi @ Q @ xi + q @ xi
            g[us(k)] += M.T @ xi
        else:
            H[xs(k), xs(k)] += Q
            H[xs(k), us(k)] += M
            H[us(k), xs(k)] += M.T
            g[xs(k)] += q
        rows = slice(k * n, (k + 1) * n)
        # A x_k + B u_k + c - x_{k+1} = 0
        Ecs[rows, us(k)] += B
        if k == 0:
            ecs[rows] += A @ xi + c
        else:
            Ecs[rows, xs(k)] += A
            ecs[rows] += c
        if k == L - 1:
            ecs[rows] -= xj
        else:
            Ecs[rows, xs(k + 1)] -= np.eye(n)
    # eliminate the constraints: w = w_p + Z y
    wp, *_ = np.linalg.lstsq(Ecs, -ecs, rcond=None)
    if np.linalg.norm(Ecs @ wp + ecs) > 1e-8 * (1 + np.linalg.norm(ecs)):
        return None
    U, s, Vt = np.linalg.svd(Ecs)
    rank = int((s > 1e-12 * s[0]).sum())
    Z = Vt[rank:].T
    if Z.shape[1] > 0:
        Hr = Z.T @ H @ Z
        gr = Z.T @ (H @ wp + g)
        y = np.linalg.solve(Hr, -gr)
        w = wp + Z @ y
    else:
        w = wp
    return 0.5 * w @ H @ w + g @ w + const


def dual_value(elem, xi, xj):
    """Evaluate an element (A, b, C, P, p) in the dual form
    max_eta 1/2 xi'P xi + p'xi - 1/2 eta'C eta - eta'(xj - A xi - b):
    the inner maximum is 1/2 d'C^+ d with d = xj - A xi - b when d lies in
    range(C), +inf otherwise (returned as None)."""
    A, b, C, P, p = elem
    d = xj - A @ xi - b
    eta, *_ = np.linalg.lstsq(C, d, rcond=None)
    if np.linalg.norm(C @ eta - d) > 1e-8 * (1 + np.linalg.norm(d)):
        return None
    return 0.5 * xi @ P @ xi + p @ xi + 0.5 * d @ eta


def dropped_constant(stages):
    """Sum of the constants -1/2 r'R^{-1}r that the dual-form element omits."""
    return sum(-0.5 * st[7] @ np.linalg.solve(st[4], st[7]) for st in stages)


# ---------------------------------------------------------------- exact ----

def fraction_solve(K, rhs):
    """Exact Gauss-Jordan elimination over the rationals (small systems)."""
    n = len(rhs)
    A = [[Fraction(K[i][j]) for j in range(n)] + [Fraction(rhs[i])] for i in range(n)]
    for col in range(n):
        piv = next(i for i in range(col, n) if A[i][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [v / pv for v in A[col]]
        for i in range(n):
            if i != col and A[i][col] != 0:
                f = A[i][col]
                A[i] = [a - f * b for a, b in zip(A[i], A[col])]
    return [A[i][n] for i in range(n)]
