"""Pins of the line-search and SQP oracle (oracle/sqp.py) against what the
mathematics fixes: the model's Jacobians against finite differences; with
linear dynamics and a quadratic cost the Gauss-Newton step is exact, so the
defects shrink as (1 - alpha) theta0 and the cost along the step is the
quadratic J0 + alpha dJ + alpha^2 (J(1) - J0 - dJ); the filter test's three
branches on hand-made cases; and the iteration on the bilinear model
converges (defects and step go to zero)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import sqp


def _model(N=12, n=6, m=3, nc=4, gamma=0.05, seed=1):
    return synth.gen_bilinear(N, n, m, nc, [seed], gamma)


def test_dynamics_jacobians_match_finite_differences():
    mdl = _model()
    rng = np.random.default_rng(0)
    x, u = rng.normal(size=6), rng.normal(size=3)
    Ax, Bu = sqp.dyn_jac(mdl, x, u)
    h = 1e-6
    for j in range(6):
        d = np.zeros(6); d[j] = h
        assert np.allclose((sqp.dyn(mdl, x + d, u) - sqp.dyn(mdl, x - d, u)) / (2 * h), Ax[:, j], atol=1e-8)
    for j in range(3):
        d = np.zeros(3); d[j] = h
        assert np.allclose((sqp.dyn(mdl, x, u + d) - sqp.dyn(mdl, x, u - d)) / (2 * h), Bu[:, j], atol=1e-8)


def test_linear_quadratic_case_is_exact():
    mdl = _model(nc=0, gamma=0.0)
    N, n, m = 12, 6, 3
    X = np.tile(mdl["xhat0"], (N + 1, 1)) + np.random.default_rng(1).normal(0, 0.1, (N + 1, n))
    U = np.zeros((N, m))
    qp = sqp.qp_of(mdl, X, U, mdl["xhat0"])
    sol = oracle.riccati(qp)
    dX, dU = sol["x"], sol["u"]
    dJ = float(np.sum(qp["q"] * dX) + np.sum(qp["r"] * dU))
    th0, J0 = sqp.theta(mdl, X, U), sqp.cost(mdl, X, U)
    J1 = sqp.cost(mdl, X + dX, U + dU)
    curv = J1 - J0 - dJ
    assert curv > 0 and dJ < 0
    for a in (0.25, 0.5, 0.75, 1.0):
        assert abs(sqp.theta(mdl, X + a * dX, U + a * dU) - (1 - a) * th0) <= 1e-12 * max(1.0, th0)
        assert abs(sqp.cost(mdl, X + a * dX, U + a * dU) - (J0 + a * dJ + a * a * curv)) <= 1e-10 * abs(J0)
    # the full step is optimal: a second subproblem at the new iterate has a zero step
    qp2 = sqp.qp_of(mdl, X + dX, U + dU, mdl["xhat0"])
    sol2 = oracle.riccati(qp2)
    assert np.abs(sol2["x"]).max() < 1e-10 and np.abs(sol2["u"]).max() < 1e-10


@pytest.mark.parametrize("case,expect", [
    # theta0 above theta_max: only a decrease of theta counts
    ((2.0, 5.0, 1.9, 9.0, 1.0, -1.0, 1.0), True), ((2.0, 5.0, 2.1, 1.0, 1.0, -1.0, 1.0), False),
    # below: Armijo on a descent direction
    ((0.5, 5.0, 9.0, 4.9, 1.0, -1.0, 1.0), True), ((0.5, 5.0, 0.1, 4.99999, 1.0, -1.0, 1.0), False),
    # below, not a descent direction: cost or theta must drop
    ((0.5, 5.0, 0.4, 6.0, 1.0, 1.0, 1.0), True), ((0.5, 5.0, 0.6, 4.0, 1.0, 1.0, 1.0), True),
    ((0.5, 5.0, 0.6, 6.0, 1.0, 1.0, 1.0), False)])
def test_filter_branches(case, expect):
    th0, J0, th, J, a, dJ, tmax = case
    assert sqp.filter_accepts(th0, J0, th, J, a, dJ, tmax, eta=1e-4) is expect


def test_iteration_converges_on_the_bilinear_model():
    mdl = _model(gamma=0.2)
    N, n, m = 12, 6, 3
    X = np.tile(mdl["xhat0"], (N + 1, 1))
    U = np.zeros((N, m))
    L = np.zeros((N + 1, n))
    alphas = []
    for _ in range(40):   # Gauss-Newton converges linearly here (the dynamics' second derivative is dropped)
        X, U, L, a = sqp.sqp_iteration(mdl, X, U, L, mdl["xhat0"], oracle.riccati, theta_max=1e-2)
        alphas.append(a)
    qp = sqp.qp_of(mdl, X, U, mdl["xhat0"])
    sol = oracle.riccati(qp)
    assert sqp.theta(mdl, X, U) < 1e-12
    assert np.abs(sol["x"]).max() < 1e-5 and np.abs(sol["u"]).max() < 1e-5
    assert alphas[-1] == 1.0
