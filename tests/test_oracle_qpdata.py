"""Pins of the QP-data builder oracle (oracle/qpdata.py), independent of its
own derivative formulas: the stage cost is written out from its definition
(Sec. II-F: 1/2 eps' W eps plus the relaxed barriers, with eps and xi linear
in (dx, du) at the linearization point) and differentiated numerically; for
linear eps and xi the Gauss-Newton blocks are the exact Hessian and the
linear terms the exact gradient.  Also: the barrier's two branches join
with continuous value, slope and curvature, its curvature is positive, and
the stage Hessian is positive definite."""
import numpy as np
import pytest

import synth
from oracle import qpdata


def _stage(seed, terminal=False, n=5, m=3, nc=4):
    d = synth.gen_qpdata(2, n, m, nc, seed)
    k = 1 if terminal else 0
    return d, k


def _cost(d, k, z, n, terminal):
    """Stage cost at (dx, du) = z, from the definitions."""
    dx = z[:n]
    e = d["e"][k] + d["Ex"][k] @ dx
    xi = d["g"][k] + d["Gx"][k] @ dx
    if not terminal:
        du = z[n:]
        e = e + d["Eu"][k] @ du
        xi = xi + d["Gu"][k] @ du
    return 0.5 * e @ d["W"][k] @ e + float(np.sum(qpdata.barrier(xi, d["mu"], d["delta"])))


@pytest.mark.parametrize("terminal", [False, True])
@pytest.mark.parametrize("seed", [[1], [2], [3]])
def test_blocks_equal_numerical_derivatives_of_the_cost(seed, terminal):
    n, m = 5, 3
    d, k = _stage(seed, terminal, n, m)
    if terminal:
        Q, _, _, q, _ = qpdata.build_stage(d["Ex"][k], d["e"][k], d["W"][k], d["Gx"][k], d["g"][k], d["mu"], d["delta"])
        H = Q
        gr = q
    else:
        Q, M, R, q, r = qpdata.build_stage(d["Ex"][k], d["e"][k], d["W"][k], d["Gx"][k], d["g"][k], d["mu"],
                                           d["delta"], d["Eu"][k], d["Gu"][k])
        H = np.block([[Q, M], [M.T, R]])
        gr = np.concatenate([q, r])
    dim = H.shape[0]
    # keep every constraint on one branch over the stencil (the barrier is
    # only C2 at xi = delta)
    h1, h2 = 1e-6, 1e-4
    z0 = np.zeros(dim)
    num_g = np.array([(_cost(d, k, z0 + h1 * np.eye(dim)[i], n, terminal) -
                       _cost(d, k, z0 - h1 * np.eye(dim)[i], n, terminal)) / (2 * h1) for i in range(dim)])
    assert np.allclose(num_g, gr, rtol=1e-6, atol=1e-6 * np.abs(gr).max()), (num_g, gr)
    num_H = np.zeros((dim, dim))
    for i in range(dim):
        for j in range(dim):
            ei, ej = h2 * np.eye(dim)[i], h2 * np.eye(dim)[j]
            num_H[i, j] = (_cost(d, k, ei + ej, n, terminal) - _cost(d, k, ei - ej, n, terminal) -
                           _cost(d, k, -ei + ej, n, terminal) + _cost(d, k, -ei - ej, n, terminal)) / (4 * h2 * h2)
    assert np.allclose(num_H, H, rtol=1e-4, atol=1e-5 * np.abs(H).max()), np.abs(num_H - H).max()


def test_barrier_branches_join_smoothly():
    mu, delta = 0.07, 0.13
    for f, tol in ((qpdata.barrier, 1e-12), (qpdata.barrier_d1, 1e-9), (qpdata.barrier_d2, 1e-9)):
        below = float(f(delta * (1 - 1e-12), mu, delta))
        at = float(f(delta, mu, delta))
        assert abs(below - at) <= tol * max(1.0, abs(at)), (f.__name__, below, at)
    xi = np.linspace(-1.0, 2.0, 301)
    assert (qpdata.barrier_d2(xi, mu, delta) > 0).all()
    # slope by differences of the value, on both branches
    for x in (-0.5, 0.05, 0.5, 1.5):
        h = 1e-6
        num = (float(qpdata.barrier(x + h, mu, delta)) - float(qpdata.barrier(x - h, mu, delta))) / (2 * h)
        assert abs(num - float(qpdata.barrier_d1(x, mu, delta))) <= 1e-6 * max(1.0, abs(num))


def test_barrier_log_branch_is_the_log_barrier():
    xi = np.array([0.3, 1.0, 4.0])
    assert np.allclose(qpdata.barrier(xi, 0.1, 0.2), -0.1 * np.log(xi))


def test_stage_hessian_positive_definite_and_batch_matches_stages():
    d = synth.gen_qp_batch(2, 6, 5, 3, 4, [7])
    out = qpdata.build(d)
    for b in range(2):
        for k in range(6):
            H = np.block([[out["Q"][b, k], out["M"][b, k]], [out["M"][b, k].T, out["R"][b, k]]])
            assert np.linalg.eigvalsh(H).min() > 0
            Q, M, R, q, r = qpdata.build_stage(d["Ex"][b, k], d["e"][b, k], d["W"][b, k], d["Gx"][b, k], d["g"][b, k],
                                               d["mu"], d["delta"], d["Eu"][b, k], d["Gu"][b, k])
            assert np.array_equal(Q, out["Q"][b, k]) and np.array_equal(r, out["r"][b, k])
        assert np.linalg.eigvalsh(out["Q"][b, 6]).min() > 0
