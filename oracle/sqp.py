"""CPU FP64 oracle of the parallel filter line search and of the SQP
iteration around the KKT solve, on a synthetic nonlinear model (test
infrastructure only: only tests/, __graft_entry__.smoke() and bench.py's
CPU-baseline leg may import it; the GPU path never does).

Paper: Amatucci, Sousa-Pinto et al., arXiv 2506.07823, Sec. II-B (the SQP
subproblem), II-E (parallel line search), II-F (Gauss-Newton blocks,
relaxed barriers, one iteration per control tick).

Model (a stand-in for the robot models, which are not available): dynamics
with a bilinear term, as in rigid-body dynamics where forces enter through
products with states,
    h(x, u) = A x + B u + c + gamma (P x) * (V u)        (* elementwise)
a tracking cost with diagonal weights and linear inequality constraints
xi = Gx x + Gu u + g0 >= 0 under the relaxed barrier of Sec. II-F,
    l_k = 1/2 sum wx_k (x_k - xr_k)^2 + 1/2 sum wu_k (u_k - ur_k)^2 + sum_j B(xi_j(x_k, u_k))
    l_N = 1/2 sum wx_N (x_N - xr_N)^2 + sum_j B(Gx_j x_N + g0_j).

Line search (Sec. II-E): the trial iterates z + alpha dz for alpha in
{2^0, ..., 2^-9}; theta(alpha) = sum_k ||x_{k+1} - h(x_k, u_k)||_2 (the
dynamics defects), J(alpha) the cost.  With theta0, J0 at alpha = 0 and
the directional derivative dJ of the cost along dz:
  theta0 > theta_max:      accept alpha if theta(alpha) < theta0;
  else if dJ < 0:          accept if J(alpha) <= J0 + eta alpha dJ (Armijo);
  else:                    accept if J(alpha) < J0 or theta(alpha) < theta0.
The largest accepted alpha is taken; none accepted gives alpha = 0.
Readings: theta sums the dynamics defects only (the initial-state
constraint is met by the full step of the QP); the multiplier update is
lam + alpha (lam_QP - lam) with lam_QP the subproblem's costates.
"""
from __future__ import annotations

import numpy as np

from oracle import qpdata

ALPHAS = tuple(2.0 ** -i for i in range(10))


def dyn(mdl, x, u):
    """h(x, u) of one stage."""
    return mdl["A"] @ x + mdl["B"] @ u + mdl["c"] + mdl["gamma"] * (mdl["P"] @ x) * (mdl["V"] @ u)


def dyn_jac(mdl, x, u):
    """(dh/dx, dh/du) of one stage."""
    Px, Vu = mdl["P"] @ x, mdl["V"] @ u
    return (mdl["A"] + mdl["gamma"] * Vu[:, None] * mdl["P"], mdl["B"] + mdl["gamma"] * Px[:, None] * mdl["V"])


def cost(mdl, X, U):
    """J of a trajectory X [N+1][n], U [N][m]."""
    N = U.shape[0]
    J = 0.0
    for k in range(N + 1):
        dx = X[k] - mdl["xr"][k]
        J += 0.5 * float(np.sum(mdl["wx"][k] * dx * dx))
        xi = mdl["Gx"] @ X[k] + mdl["g0"]
        if k < N:
            du = U[k] - mdl["ur"][k]
            J += 0.5 * float(np.sum(mdl["wu"][k] * du * du))
            xi = xi + mdl["Gu"] @ U[k]
        J += float(np.sum(qpdata.barrier(xi, mdl["mu"], mdl["delta"])))
    return J


def theta(mdl, X, U):
    """Dynamics violation: sum of the 2-norms of the stage defects."""
    return float(sum(np.linalg.norm(X[k + 1] - dyn(mdl, X[k], U[k])) for k in range(U.shape[0])))


def qp_of(mdl, X, U, xhat0):
    """The subproblem of Sec. II-B at iterate (X, U): dynamics Jacobians and
    defects, Gauss-Newton blocks of the cost (tracking residual with
    selection Jacobians, weights diag(wx, wu)), x0 = xhat0 - X_0."""
    N, m = U.shape
    n = X.shape[1]
    p = n + m
    A = np.zeros((N, n, n)); B = np.zeros((N, n, m)); c = np.zeros((N, n))
    Q = np.zeros((N + 1, n, n)); M = np.zeros((N, n, m)); R = np.zeros((N, m, m))
    q = np.zeros((N + 1, n)); r = np.zeros((N, m))
    Ex = np.zeros((p, n)); Ex[:n] = np.eye(n)
    Eu = np.zeros((p, m)); Eu[n:] = np.eye(m)
    for k in range(N + 1):
        e = np.concatenate([X[k] - mdl["xr"][k], (U[k] - mdl["ur"][k]) if k < N else np.zeros(m)])
        W = np.diag(np.concatenate([mdl["wx"][k], mdl["wu"][k] if k < N else np.zeros(m)]))
        g = mdl["Gx"] @ X[k] + mdl["g0"] + (mdl["Gu"] @ U[k] if k < N else 0.0)
        if k < N:
            A[k], B[k] = dyn_jac(mdl, X[k], U[k])
            c[k] = dyn(mdl, X[k], U[k]) - X[k + 1]
            Q[k], M[k], R[k], q[k], r[k] = qpdata.build_stage(Ex, e, W, mdl["Gx"], g, mdl["mu"], mdl["delta"], Eu,
                                                              mdl["Gu"])
        else:
            Q[k], _, _, q[k], _ = qpdata.build_stage(Ex, e, W, mdl["Gx"], g, mdl["mu"], mdl["delta"])
    return {"A": A, "B": B, "c": c, "Q": Q, "R": R, "M": M, "q": q, "r": r, "x0": xhat0 - X[0]}


def line_search(mdl, X, U, dX, dU, dJ, theta_max, eta=1e-4):
    """Filter line search of Sec. II-E over ALPHAS; returns (alpha, index of
    alpha or -1, theta per alpha, J per alpha, theta0, J0)."""
    th0, J0 = theta(mdl, X, U), cost(mdl, X, U)
    ths = [theta(mdl, X + a * dX, U + a * dU) for a in ALPHAS]
    Js = [cost(mdl, X + a * dX, U + a * dU) for a in ALPHAS]
    for i, a in enumerate(ALPHAS):
        if filter_accepts(th0, J0, ths[i], Js[i], a, dJ, theta_max, eta):
            return a, i, ths, Js, th0, J0
    return 0.0, -1, ths, Js, th0, J0


def filter_accepts(th0, J0, th, J, alpha, dJ, theta_max, eta=1e-4):
    """The acceptance test of Sec. II-E for one trial step."""
    if th0 > theta_max:
        return th < th0
    if dJ < 0:
        return J <= J0 + eta * alpha * dJ
    return J < J0 or th < th0


def sqp_iteration(mdl, X, U, L, xhat0, solve, theta_max, eta=1e-4):
    """One SQP iteration: subproblem, its solve by `solve` (a function of a
    problem dict returning dict x, u, lam, e.g. oracle.riccati), the
    directional derivative of the cost along the step from the subproblem's
    gradient, line search and update.  Returns (X, U, L, alpha)."""
    qp = qp_of(mdl, X, U, xhat0)
    sol = solve(qp)
    dX, dU = sol["x"], sol["u"]
    dJ = float(np.sum(qp["q"] * dX) + np.sum(qp["r"] * dU))
    a, _, _, _, _, _ = line_search(mdl, X, U, dX, dU, dJ, theta_max, eta)
    return X + a * dX, U + a * dU, L + a * (sol["lam"] - L), a
