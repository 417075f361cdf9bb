"""Pins of the CPU FP64 oracle against things other than itself.

Each test fixes the oracle to something the paper or the mathematics fixes:
  * exact hand-derived values (tests/golden/scalar_hand.txt),
  * exact rational solves of the KKT system built from the QP statement,
  * dense LAPACK solves of that KKT system (brute force, tiny sizes),
  * textbook special cases (scalar Riccati, N = 1, B = 0, the DARE limit),
  * brute-force conditional value functions (min over intermediate states),
  * invariants (residual, symmetry/definiteness, optimality, linearity,
    associativity of the combine, complete suffixes).
"""
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import synth
from tests import pinlib

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    a = np.asarray(a, dtype=float); b = np.asarray(b, dtype=float)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def scalar_prob(a, b, c, Q0, R, M, Q1, q0, r, q1, xinit):
    arr = lambda v: np.array(v, dtype=float)
    return dict(A=arr([[[a]]]), B=arr([[[b]]]), c=arr([[c]]), Q=arr([[[Q0]], [[Q1]]]),
                R=arr([[[R]]]), M=arr([[[M]]]), q=arr([[q0], [q1]]), r=arr([[r]]), x0=arr([xinit]))


def load_golden():
    cases = []
    with open(os.path.join(GOLDEN, "scalar_hand.txt")) as f:
        for line in f:
            if line.startswith("case"):
                kv = dict(tok.split("=") for tok in line.split()[1:])
                cases.append({k: Fraction(v) for k, v in kv.items()})
    return cases


# ------------------------------------------------------------ exact values --

@pytest.mark.parametrize("case", load_golden(), ids=lambda c: f"a{c['a']}b{c['b']}")
def test_hand_derived_scalar_cases(oracle_lib, case):
    f = {k: float(v) for k, v in case.items()}
    prob = scalar_prob(f["a"], f["b"], f["c"], f["Q0"], f["R"], f["M"], f["Q1"], f["q0"], f["r"],
                       f["q1"], f["xinit"])
    out = oracle_lib.riccati(prob, want_factors=True)
    assert out["x"][0, 0] == pytest.approx(f["x0"], abs=1e-14)
    assert out["x"][1, 0] == pytest.approx(f["x1"], abs=1e-14)
    assert out["u"][0, 0] == pytest.approx(f["u0"], abs=1e-14)
    assert out["lam"][0, 0] == pytest.approx(f["lam0"], abs=1e-14)
    assert out["lam"][1, 0] == pytest.approx(f["lam1"], abs=1e-14)
    assert out["P"][0, 0, 0] == pytest.approx(f["P0"], abs=1e-14)
    assert out["p"][0, 0] == pytest.approx(f["p0"], abs=1e-14)


def _int_prob(seed, N, n, m):
    """Small-integer problem whose stage Hessians are positive definite."""
    rng = np.random.default_rng(seed)
    A = rng.integers(-2, 3, (N, n, n)).astype(float)
    B = rng.integers(-2, 3, (N, n, m)).astype(float)
    c = rng.integers(-2, 3, (N, n)).astype(float)
    Q = np.stack([np.eye(n) * (n + 2) + np.triu(np.ones((n, n)), 1) + np.triu(np.ones((n, n)), 1).T
                  for _ in range(N + 1)])
    R = np.stack([np.eye(m) * (m + 1) + 0.0 for _ in range(N)])
    M = rng.integers(0, 2, (N, n, m)).astype(float)
    q = rng.integers(-3, 4, (N + 1, n)).astype(float)
    r = rng.integers(-3, 4, (N, m)).astype(float)
    x0 = rng.integers(-3, 4, n).astype(float)
    return dict(A=A, B=B, c=c, Q=Q, R=R, M=M, q=q, r=r, x0=x0)


@pytest.mark.parametrize("seed,N,n,m", [(0, 2, 2, 1), (1, 3, 2, 2), (2, 2, 3, 1)])
def test_exact_rational_kkt(oracle_lib, seed, N, n, m):
    """KKT system of the QP solved exactly over the rationals."""
    prob = _int_prob(seed, N, n, m)
    for k in range(N):  # stage Hessian must be PD for the test to be meaningful
        Hs = np.block([[prob["Q"][k], prob["M"][k]], [prob["M"][k].T, prob["R"][k]]])
        assert np.linalg.eigvalsh(Hs)[0] > 0
    K, rhs = pinlib.dense_kkt(prob)
    z = np.array([float(v) for v in pinlib.fraction_solve(K.tolist(), rhs.tolist())])
    nx, nu, nz = pinlib.unknown_layout(N, n, m)
    out = oracle_lib.riccati(prob)
    assert rel(out["x"].ravel(), z[:nx]) < 1e-13
    assert rel(out["u"].ravel(), z[nx:nz]) < 1e-13
    assert rel(out["lam"].ravel(), z[nz:]) < 1e-13


# ------------------------------------------------------ dense brute force --

SIZES = [(1, 1, 1), (4, 2, 1), (16, 4, 2), (7, 3, 3), (9, 5, 1), (6, 6, 4), (12, 3, 2)]


@pytest.mark.parametrize("N,n,m", SIZES)
def test_dense_kkt_matches(oracle_lib, N, n, m):
    prob = synth.gen_rand(N, n, m, seed=[101, N, n, m])
    xd, ud, ld = pinlib.dense_solve(prob)
    out = oracle_lib.riccati(prob)
    assert rel(out["x"], xd) < 1e-11
    assert rel(out["u"], ud) < 1e-11
    assert rel(out["lam"], ld) < 1e-11


def test_dense_kkt_matches_tiny_config(oracle_lib):
    prob = synth.gen_c1(0)
    xd, ud, ld = pinlib.dense_solve(prob)
    out = oracle_lib.riccati(prob)
    for a, b in ((out["x"], xd), (out["u"], ud), (out["lam"], ld)):
        assert rel(a, b) < 1e-11


@pytest.mark.parametrize("N,n,m", [(5, 3, 2), (8, 4, 4)])
def test_value_function_from_dense(oracle_lib, N, n, m):
    """lam_0 is affine in x0 with slope P_0 and offset p_0 (lam = P x + p):
    probe the dense KKT solve at x0 = 0 and x0 = e_j."""
    prob = synth.gen_rand(N, n, m, seed=[7, N])
    out = oracle_lib.riccati(prob, want_factors=True)
    p0 = dict(prob); p0["x0"] = np.zeros(n)
    _, _, l0 = pinlib.dense_solve(p0)
    P = np.zeros((n, n))
    for j in range(n):
        pj = dict(prob); pj["x0"] = np.eye(n)[j]
        _, _, lj = pinlib.dense_solve(pj)
        P[:, j] = lj[0] - l0[0]
    assert rel(out["P"][0], P) < 1e-10
    assert rel(out["p"][0], l0[0]) < 1e-10


def test_residual_function_is_the_kkt_operator(oracle_lib):
    """For arbitrary (x, u, lam) the oracle's residual equals K z - rhs of the
    dense KKT system (reordered into the oracle's block order)."""
    N, n, m = 5, 3, 2
    prob = synth.gen_rand(N, n, m, seed=11)
    K, rhs = pinlib.dense_kkt(prob)
    rng = np.random.default_rng(3)
    x = rng.normal(size=(N + 1, n)); u = rng.normal(size=(N, m)); lam = rng.normal(size=(N + 1, n))
    z = np.concatenate([x.ravel(), u.ravel(), lam.ravel()])
    dense = K @ z - rhs
    nx, nu, nz = pinlib.unknown_layout(N, n, m)
    stat_x, stat_u, feas = dense[:nx], dense[nx:nz], dense[nz:]
    res, nr, nb = oracle_lib.kkt_residual(prob, x, u, lam)
    # oracle order: r_init (n) = x_0 - x0, r_dyn (N n), r_x ((N+1) n), r_u (N m)
    # dense feasibility rows are E z + e = -x_0 + x0, A x + B u + c - x'
    assert np.allclose(res[:n], -feas[:n], atol=1e-12)
    assert np.allclose(res[n:n + N * n], feas[n:], atol=1e-12)
    assert np.allclose(res[n + N * n:n + N * n + nx], stat_x, atol=1e-12)
    assert np.allclose(res[n + N * n + nx:], stat_u, atol=1e-12)
    assert nr == pytest.approx(np.linalg.norm(res))
    ref = np.sqrt(sum(np.sum(prob[k] ** 2) for k in ("x0", "c", "q", "r")))
    assert nb == pytest.approx(ref)


# ------------------------------------------------------ textbook specials --

def test_scalar_riccati_textbook(oracle_lib):
    """n = m = 1, time-varying: P <- q + a^2 P - (s + a b P)^2 / (rho + b^2 P)."""
    rng = np.random.default_rng(5)
    N = 9
    a = rng.uniform(0.5, 1.5, N); b = rng.uniform(-1, 1, N); cc = rng.normal(size=N)
    qq = rng.uniform(0.5, 2, N + 1); rho = rng.uniform(0.5, 2, N); s = rng.uniform(-0.2, 0.2, N)
    lq = rng.normal(size=N + 1); lr = rng.normal(size=N)
    prob = dict(A=a.reshape(N, 1, 1), B=b.reshape(N, 1, 1), c=cc.reshape(N, 1),
                Q=qq.reshape(N + 1, 1, 1), R=rho.reshape(N, 1, 1), M=s.reshape(N, 1, 1),
                q=lq.reshape(N + 1, 1), r=lr.reshape(N, 1), x0=np.array([0.7]))
    out = oracle_lib.riccati(prob, want_factors=True)
    P, p = qq[N], lq[N]
    Ps, ps = [P], [p]
    for k in reversed(range(N)):
        g = rho[k] + b[k] ** 2 * P
        hx = s[k] + a[k] * b[k] * P
        v = p + P * cc[k]
        hu = b[k] * v + lr[k]
        P, p = qq[k] + a[k] ** 2 * P - hx ** 2 / g, lq[k] + a[k] * v - hx * hu / g
        Ps.append(P); ps.append(p)
    Ps, ps = Ps[::-1], ps[::-1]
    assert rel(out["P"].ravel(), Ps) < 1e-13
    assert rel(out["p"].ravel(), ps) < 1e-13


def test_horizon_one_closed_form(oracle_lib):
    prob = synth.gen_rand(1, 4, 3, seed=21)
    A, B, c, Q, R, M, q, r = (prob[k] for k in ("A", "B", "c", "Q", "R", "M", "q", "r"))
    x0 = prob["x0"]
    u0 = -np.linalg.solve(R[0] + B[0].T @ Q[1] @ B[0],
                          M[0].T @ x0 + r[0] + B[0].T @ (Q[1] @ (A[0] @ x0 + c[0]) + q[1]))
    x1 = A[0] @ x0 + B[0] @ u0 + c[0]
    l1 = Q[1] @ x1 + q[1]
    l0 = Q[0] @ x0 + M[0] @ u0 + q[0] + A[0].T @ l1
    out = oracle_lib.riccati(prob)
    assert rel(out["u"][0], u0) < 1e-13
    assert rel(out["x"][1], x1) < 1e-13
    assert rel(out["lam"], np.stack([l0, l1])) < 1e-13


def test_zero_input_matrix(oracle_lib):
    """B = 0: the state is the open-loop affine rollout and every control
    minimizes its own stage cost, u_k = -R_k^{-1}(M_k' x_k + r_k)."""
    prob = synth.gen_rand(8, 4, 2, seed=33)
    prob["B"] = np.zeros_like(prob["B"])
    out = oracle_lib.riccati(prob)
    x = [prob["x0"]]
    for k in range(8):
        x.append(prob["A"][k] @ x[-1] + prob["c"][k])
    x = np.stack(x)
    u = np.stack([-np.linalg.solve(prob["R"][k], prob["M"][k].T @ x[k] + prob["r"][k]) for k in range(8)])
    assert rel(out["x"], x) < 1e-13
    assert rel(out["u"], u) < 1e-13


@pytest.mark.parametrize("n,m,cross", [(4, 2, 0.0), (6, 3, 0.3)])
def test_dare_limit(oracle_lib, n, m, cross):
    """Long time-invariant horizon: P_0 converges to the stabilizing solution
    of the discrete algebraic Riccati equation (with cross term s = M)."""
    rng = np.random.default_rng([n, m])
    A = np.eye(n) + 0.3 * rng.normal(size=(n, n)) / np.sqrt(n)
    B = rng.normal(size=(n, m))
    G = rng.normal(size=(n, n)); Q = G @ G.T / n + np.eye(n)
    H = rng.normal(size=(m, m)); R = H @ H.T / m + np.eye(m)
    M = rng.normal(size=(n, m))
    M *= cross * np.sqrt(np.linalg.eigvalsh(Q)[0] * np.linalg.eigvalsh(R)[0]) / np.linalg.norm(M, 2)
    N = 400
    prob = dict(A=np.broadcast_to(A, (N, n, n)).copy(), B=np.broadcast_to(B, (N, n, m)).copy(),
                c=np.zeros((N, n)), Q=np.broadcast_to(Q, (N + 1, n, n)).copy(),
                R=np.broadcast_to(R, (N, m, m)).copy(), M=np.broadcast_to(M, (N, n, m)).copy(),
                q=np.zeros((N + 1, n)), r=np.zeros((N, m)), x0=np.ones(n))
    out = oracle_lib.riccati(prob, want_factors=True)
    X = scipy.linalg.solve_discrete_are(A, B, Q, R, s=M)
    assert rel(out["P"][0], X) < 1e-8


# --------------------------------------------------------------- invariants --

@pytest.mark.parametrize("gen", ["c1", "c2_25", "rand"])
def test_invariants(oracle_lib, gen):
    if gen == "c1":
        prob = synth.gen_c1(3)
    elif gen == "c2_25":
        prob = synth.gen_c2(25, 1)
    else:
        prob = synth.gen_rand(20, 5, 3, seed=9)
    N, n, m = prob["B"].shape
    out = oracle_lib.riccati(prob, want_factors=True)
    assert oracle_lib.rel_kkt_residual(prob, out["x"], out["u"], out["lam"]) < 1e-13
    for k in range(N + 1):
        P = out["P"][k]
        assert np.allclose(P, P.T, rtol=0, atol=1e-12 * np.abs(P).max())
        np.linalg.cholesky(P)
        if k < N:   # P_k dominates the one-stage Schur complement Q - M R^{-1} M'
            S = prob["Q"][k] - prob["M"][k] @ np.linalg.solve(prob["R"][k], prob["M"][k].T)
            assert np.linalg.eigvalsh(P - S)[0] > -1e-10 * np.abs(P).max()
    # optimality: any feasible perturbation raises the QP cost
    J0 = pinlib.qp_cost(prob, out["x"], out["u"])
    rng = np.random.default_rng(1)
    for _ in range(5):
        u = out["u"] + 1e-2 * rng.normal(size=out["u"].shape)
        x = [prob["x0"]]
        for k in range(N):
            x.append(prob["A"][k] @ x[-1] + prob["B"][k] @ u[k] + prob["c"][k])
        assert pinlib.qp_cost(prob, np.stack(x), u) > J0


def test_linearity_in_vector_data(oracle_lib):
    """With the matrices fixed, (x, u, lam) is linear in (x0, c, q, r)."""
    N, n, m = 10, 4, 3
    base = synth.gen_rand(N, n, m, seed=41)
    rng = np.random.default_rng(2)

    def with_vec(seed):
        g = np.random.default_rng(seed)
        p = dict(base)
        for k in ("x0", "c", "q", "r"):
            p[k] = g.normal(size=base[k].shape)
        return p

    p1, p2 = with_vec(1), with_vec(2)
    al, be = 0.7, -1.3
    p3 = dict(base)
    for k in ("x0", "c", "q", "r"):
        p3[k] = al * p1[k] + be * p2[k]
    o1, o2, o3 = (oracle_lib.riccati(p) for p in (p1, p2, p3))
    for f in ("x", "u", "lam"):
        assert rel(o3[f], al * o1[f] + be * o2[f]) < 1e-12
    del rng


# ------------------------------------------- conditional value functions --

def _stages(prob, lo, hi):
    import oracle
    return [oracle.stage(prob, k) for k in range(lo, hi)]


@pytest.mark.parametrize("n,m", [(3, 3), (4, 2), (5, 1)])
def test_element_is_one_stage_cvf(oracle_lib, n, m):
    """eq. (initialization): the dual-form element equals the brute-force
    minimum of the stage cost over u subject to the dynamics (up to the
    dropped constant), at reachable (x_k, x_{k+1})."""
    prob = synth.gen_rand(1, n, m, seed=[55, n, m])
    st = _stages(prob, 0, 1)
    e = oracle_lib.element(*st[0])
    rng = np.random.default_rng(8)
    for _ in range(4):
        xi = rng.normal(size=n)
        u = rng.normal(size=m)
        xj = st[0][0] @ xi + st[0][1] @ u + st[0][2]
        brute = pinlib.segment_value(st, xi, xj)
        dual = pinlib.dual_value(e, xi, xj)
        assert dual is not None
        assert dual + pinlib.dropped_constant(st) == pytest.approx(brute, rel=1e-11, abs=1e-11)
    if m < n:   # off the reachable set the dual form is +inf as well
        xj = rng.normal(size=n)
        assert pinlib.segment_value(st, xi, xj) is None
        assert pinlib.dual_value(e, xi, xj) is None


@pytest.mark.parametrize("L,n,m", [(2, 3, 3), (2, 3, 2), (3, 4, 2), (4, 5, 2), (3, 6, 2)])
def test_combine_is_segment_cvf(oracle_lib, L, n, m):
    """eq. (combination_rule): folding the one-stage elements of a segment
    with the combine gives the brute-force conditional value function of the
    whole segment (the first element's C may be singular)."""
    prob = synth.gen_rand(L, n, m, seed=[66, L, n, m])
    st = _stages(prob, 0, L)
    es = [oracle_lib.element(*s) for s in st]
    folds = {"left": es[0], "right": es[-1]}
    for e in es[1:]:
        folds["left"] = oracle_lib.combine(folds["left"], e)
    for e in reversed(es[:-1]):
        folds["right"] = oracle_lib.combine(e, folds["right"])
    # The dual form keeps no constant term, and minimizing over the shared
    # state creates one, so the two functions agree up to one common offset.
    rng = np.random.default_rng(9)
    offsets = {k: [] for k in folds}
    scale = 0.0
    for _ in range(6):
        xi = rng.normal(size=n)
        us = rng.normal(size=(L, m))
        x = xi
        for k in range(L):
            x = st[k][0] @ x + st[k][1] @ us[k] + st[k][2]
        xj = x + (rng.normal(size=n) if L * m >= n else 0.0)
        brute = pinlib.segment_value(st, xi, xj)
        assert brute is not None
        scale = max(scale, abs(brute))
        for key, agg in folds.items():
            dual = pinlib.dual_value(agg, xi, xj)
            assert dual is not None
            offsets[key].append(brute - dual)
    for key, off in offsets.items():
        off = np.array(off)
        assert np.abs(off - off[0]).max() < 1e-9 * max(scale, 1.0), key
    assert offsets["left"][0] == pytest.approx(offsets["right"][0], rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("n,m", [(3, 1), (4, 4), (6, 2)])
def test_combine_associative(oracle_lib, n, m):
    prob = synth.gen_rand(3, n, m, seed=[77, n, m])
    e1, e2, e3 = (oracle_lib.element(*oracle_lib.stage(prob, k)) for k in range(3))
    left = oracle_lib.combine(oracle_lib.combine(e1, e2), e3)
    right = oracle_lib.combine(e1, oracle_lib.combine(e2, e3))
    for a, b in zip(left, right):
        assert rel(a, b) < 1e-12


@pytest.mark.parametrize("gen", ["c1", "rand"])
def test_suffix_fold_is_value_function(oracle_lib, gen):
    """Sec. II-D: the suffix e_k (x) ... (x) e_N (terminal element last)
    carries A = C = b = 0 exactly and its (P, p) is the value function of
    eq. (lqr)."""
    prob = synth.gen_c1(1) if gen == "c1" else synth.gen_rand(12, 5, 2, seed=88)
    N, n, m = prob["B"].shape
    ref = oracle_lib.riccati(prob, want_factors=True)
    s = oracle_lib.terminal_element(prob["Q"][N], prob["q"][N])
    for k in reversed(range(N)):
        s = oracle_lib.combine(oracle_lib.element(*oracle_lib.stage(prob, k)), s)
        A, b, C, P, p = s
        assert not A.any() and not b.any() and not C.any()
        assert rel(P, ref["P"][k]) < 1e-12
        assert rel(p, ref["p"][k]) < 1e-12


def test_suffix_tree_schedule(oracle_lib):
    """Any association order of the suffix gives the same value function
    (balanced tree vs sequential fold)."""
    prob = synth.gen_rand(11, 4, 2, seed=99)
    N = 11
    es = [oracle_lib.element(*oracle_lib.stage(prob, k)) for k in range(N)]
    es.append(oracle_lib.terminal_element(prob["Q"][N], prob["q"][N]))

    def tree(lo, hi):
        if hi - lo == 1:
            return es[lo]
        mid = (lo + hi) // 2
        return oracle_lib.combine(tree(lo, mid), tree(mid, hi))

    ref = oracle_lib.riccati(prob, want_factors=True)
    for k in (0, 3, 7):
        t = tree(k, N + 1)
        assert rel(t[3], ref["P"][k]) < 1e-12
        assert rel(t[4], ref["p"][k]) < 1e-12


def test_affine_scan_is_rollout(oracle_lib):
    """Composition of closed-loop affine maps reproduces the sequential
    rollout; it is associative; the initial map with zero matrix makes every
    prefix's matrix zero."""
    rng = np.random.default_rng(12)
    n, N = 4, 6
    Ms = rng.normal(size=(N, n, n)) * 0.5
    vs = rng.normal(size=(N, n))
    x0 = rng.normal(size=n)
    xs = [x0]
    for k in range(N):
        xs.append(Ms[k] @ xs[-1] + vs[k])
    acc = (np.zeros((n, n)), Ms[0] @ x0 + vs[0])
    assert rel(acc[1], xs[1]) < 1e-14
    for k in range(1, N):
        acc = oracle_lib.affine_combine(acc, (Ms[k], vs[k]))
        assert not acc[0].any()
        assert rel(acc[1], xs[k + 1]) < 1e-13
    f = [(Ms[k], vs[k]) for k in range(3)]
    l = oracle_lib.affine_combine(oracle_lib.affine_combine(f[0], f[1]), f[2])
    r = oracle_lib.affine_combine(f[0], oracle_lib.affine_combine(f[1], f[2]))
    assert rel(l[0], r[0]) < 1e-13 and rel(l[1], r[1]) < 1e-13
    full = l[0] @ x0 + l[1]
    assert rel(full, Ms[2] @ (Ms[1] @ (Ms[0] @ x0 + vs[0]) + vs[1]) + vs[2]) < 1e-13


def test_batch_driver_matches_single(oracle_lib):
    probs = synth.gen_batch(lambda i: synth.gen_rand(6, 3, 2, seed=[5, i]), 7, dtype=np.float64)
    x, u, lam, st = oracle_lib.riccati_batch(probs, nthreads=3)
    assert not st.any()
    for b in range(7):
        o = oracle_lib.riccati(synth.instance(probs, b))
        assert np.array_equal(o["x"], x[b]) and np.array_equal(o["u"], u[b])
        assert np.array_equal(o["lam"], lam[b])
