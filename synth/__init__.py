"""Seeded synthetic LQR-KKT inputs shaped like the paper's legged-robot QPs.

This module draws inputs only: it holds none of the solver's arithmetic, so
both the GPU path's tests/benchmark and the CPU oracle can use it.  The paper
releases no QP data (its QPs come from linearizing Go2 SRBD / whole-body
models in MuJoCo XLA), so seeded random problems with the shapes and value
distributions of Sec. III / IV stand in for them:

  c1   N=16, n=4, m=2 (tiny FP64 case)
  c2   n=m=12 (SRBD-like: 13-dim state with the quaternion reduced to 12),
       N in {25, 50, 100, 200}, dt = 0.02
  c3   n=36, m=12, N=100 (whole-body-like), batch of independent instances
  c4   n=m=192 (16 SRBD robots in one centralized problem), N=50
  rand generic well-conditioned problems of any size for tests
  c5   serving mix: clients (robots) whose requests share the client's
       matrices while x0 takes a random walk, N(0, 1e-2) per request

Every instance is drawn from ``numpy.random.default_rng([cfg_id, size_idx,
instance])`` (PCG64) in the fixed order A, B, c, Q, R, M, q, r, x0, each over
all stages at once.  N(0, s) means standard deviation s; U[a, b] uniform.
The returned arrays are float64, row-major, stage-major:
  A[N][n][n] B[N][n][m] c[N][n] Q[N+1][n][n] R[N][m][m] M[N][n][m]
  q[N+1][n] r[N][m] x0[n]
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

FIELDS = ("A", "B", "c", "Q", "R", "M", "q", "r", "x0")

C2_HORIZONS = (25, 50, 100, 200)


def field_shapes(N: int, n: int, m: int) -> dict:
    return {
        "A": (N, n, n), "B": (N, n, m), "c": (N, n), "Q": (N + 1, n, n),
        "R": (N, m, m), "M": (N, n, m), "q": (N + 1, n), "r": (N, m), "x0": (n,),
    }


def _diag_stack(d: np.ndarray) -> np.ndarray:
    """[K][n] diagonals -> [K][n][n] dense diagonal matrices."""
    K, n = d.shape
    out = np.zeros((K, n, n))
    idx = np.arange(n)
    out[:, idx, idx] = d
    return out


def _clip_cross(M: np.ndarray, Qd: np.ndarray, Rd: np.ndarray) -> np.ndarray:
    """Scale each stage's cross term so that 0.9 * sqrt(lmin(Q) lmin(R))
    bounds its spectral norm; then Q - M R^{-1} M' stays positive definite
    (Q, R are diagonal here so their extreme eigenvalues are the diagonals'
    extremes)."""
    out = M.copy()
    for k in range(M.shape[0]):
        nrm = np.linalg.norm(M[k], 2)
        if nrm > 0:
            bound = 0.9 * np.sqrt(Qd[k].min() * Rd[k].min())
            out[k] *= min(1.0, bound / nrm)
    return out


def _sparse(rng, shape, density, std):
    mask = rng.random(shape) < density
    vals = rng.normal(0.0, std, shape)
    return np.where(mask, vals, 0.0)


def gen_c1_like(N: int, n: int, m: int, seed, dt: float = 0.01) -> dict:
    """Distributions of the tiny FP64 case: A = I + dt G with G ~ N(0, 1)
    dense, B ~ N(0, 0.1), c ~ N(0, 1e-3), Q = diag U[0.1, 10], R = diag
    U[0.01, 1], M = 0, q, r ~ N(0, 1), x0 ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    A = np.eye(n) + dt * rng.normal(0.0, 1.0, (N, n, n))
    B = rng.normal(0.0, 0.1, (N, n, m))
    c = rng.normal(0.0, 1e-3, (N, n))
    Q = _diag_stack(rng.uniform(0.1, 10.0, (N + 1, n)))
    R = _diag_stack(rng.uniform(0.01, 1.0, (N, m)))
    M = np.zeros((N, n, m))
    q = rng.normal(0.0, 1.0, (N + 1, n))
    r = rng.normal(0.0, 1.0, (N, m))
    x0 = rng.normal(0.0, 1.0, n)
    return dict(A=A, B=B, c=c, Q=Q, R=R, M=M, q=q, r=r, x0=x0)


def gen_c1(instance: int = 0) -> dict:
    return gen_c1_like(16, 4, 2, [1, 0, instance], dt=0.01)


def gen_c2(N: int, instance: int = 0, n: int = 12, m: int = 12, seed=None) -> dict:
    """SRBD-shaped: A = I + dt F, dt = 0.02, F with 30 % nonzeros ~ N(0, 1);
    B ~ N(0, dt); Q = diag U[1, 100]; R = diag U[1e-3, 1e-1]; M ~ N(0, 1e-3)
    clipped; c ~ N(0, 1e-3); q, r ~ N(0, 1); x0 ~ N(0, 0.1)."""
    dt = 0.02
    if seed is None:
        size_idx = C2_HORIZONS.index(N) if N in C2_HORIZONS else N
        seed = [2, size_idx, instance]
    rng = np.random.default_rng(seed)
    A = np.eye(n) + dt * _sparse(rng, (N, n, n), 0.3, 1.0)
    B = rng.normal(0.0, dt, (N, n, m))
    c = rng.normal(0.0, 1e-3, (N, n))
    Qd = rng.uniform(1.0, 100.0, (N + 1, n))
    Rd = rng.uniform(1e-3, 1e-1, (N, m))
    M = _clip_cross(rng.normal(0.0, 1e-3, (N, n, m)), Qd[:N], Rd)
    q = rng.normal(0.0, 1.0, (N + 1, n))
    r = rng.normal(0.0, 1.0, (N, m))
    x0 = rng.normal(0.0, 0.1, n)
    return dict(A=A, B=B, c=c, Q=_diag_stack(Qd), R=_diag_stack(Rd), M=M, q=q, r=r, x0=x0)


def gen_c3(instance: int, N: int = 100, n: int = 36, m: int = 12) -> dict:
    """Whole-body-shaped: the tiny case's distributions at n=36, m=12, N=100
    with dt = 0.01."""
    return gen_c1_like(N, n, m, [3, 0, instance], dt=0.01)


def gen_c4(instance: int, N: int = 50, robots: int = 16, nr: int = 12) -> dict:
    """Centralized multi-robot: block-diagonal A = I + dt F and B ~ N(0, dt)
    per robot (SRBD-like blocks, dt = 0.02), plus off-diagonal-block entries
    that are nonzero with probability 0.05 and ~ N(0, 1e-3) in both A and B;
    Q, R, M, c, q, r, x0 drawn as in the SRBD case (M dense, clipped)."""
    dt = 0.02
    n = m = robots * nr
    rng = np.random.default_rng([4, 0, instance])
    blk = np.kron(np.eye(robots), np.ones((nr, nr))) > 0
    A = np.eye(n) + dt * _sparse(rng, (N, n, n), 0.3, 1.0)
    A = np.where(blk, A, _sparse(rng, (N, n, n), 0.05, 1e-3))
    B = np.where(blk, rng.normal(0.0, dt, (N, n, m)), _sparse(rng, (N, n, m), 0.05, 1e-3))
    c = rng.normal(0.0, 1e-3, (N, n))
    Qd = rng.uniform(1.0, 100.0, (N + 1, n))
    Rd = rng.uniform(1e-3, 1e-1, (N, m))
    M = _clip_cross(rng.normal(0.0, 1e-3, (N, n, m)), Qd[:N], Rd)
    q = rng.normal(0.0, 1.0, (N + 1, n))
    r = rng.normal(0.0, 1.0, (N, m))
    x0 = rng.normal(0.0, 0.1, n)
    return dict(A=A, B=B, c=c, Q=_diag_stack(Qd), R=_diag_stack(Rd), M=M, q=q, r=r, x0=x0)


def gen_rand(N: int, n: int, m: int, seed, cross: float = 0.1, dense_q: bool = True,
             a_scale: float = 0.3, b_scale: float = 0.5) -> dict:
    """Generic test problem: dense SPD Q and R, a cross term scaled so the
    stage Hessian [[Q, M], [M', R]] stays positive definite, and moderately
    contracting/expanding dynamics."""
    rng = np.random.default_rng(seed)
    A = np.eye(n) + a_scale * rng.normal(0.0, 1.0, (N, n, n)) / np.sqrt(n)
    B = b_scale * rng.normal(0.0, 1.0, (N, n, m))
    c = rng.normal(0.0, 0.1, (N, n))
    if dense_q:
        G = rng.normal(0.0, 1.0, (N + 1, n, n))
        Q = np.einsum("kij,klj->kil", G, G) / n + np.eye(n)
        H = rng.normal(0.0, 1.0, (N, m, m))
        R = np.einsum("kij,klj->kil", H, H) / m + 0.5 * np.eye(m)
    else:
        Q = _diag_stack(rng.uniform(0.5, 2.0, (N + 1, n)))
        R = _diag_stack(rng.uniform(0.5, 2.0, (N, m)))
    M = rng.normal(0.0, 1.0, (N, n, m))
    for k in range(N):
        lq = np.linalg.eigvalsh(Q[k])[0]
        lr = np.linalg.eigvalsh(R[k])[0]
        nrm = np.linalg.norm(M[k], 2)
        M[k] *= cross * np.sqrt(lq * lr) / max(nrm, 1e-300)
    q = rng.normal(0.0, 1.0, (N + 1, n))
    r = rng.normal(0.0, 1.0, (N, m))
    x0 = rng.normal(0.0, 1.0, n)
    return dict(A=A, B=B, c=c, Q=Q, R=R, M=M, q=q, r=r, x0=x0)


def gen_c5_clients(n_clients: int = 40) -> list:
    """Client population of the serving mix, in the request proportions
    60 % SRBD-shaped (n = m = 12, N in {25, 50, 100} equally), 30 %
    whole-body-shaped (n = 36, m = 12, N in {50, 100}) and 10 % multi-robot
    (n = m = 192, N = 50); every client issues requests at the same rate.
    Returns a list of (model dict, x0 walk seed)."""
    kinds = []
    n_mr = max(1, round(0.1 * n_clients))
    n_wb = max(1, round(0.3 * n_clients))
    n_sr = n_clients - n_mr - n_wb
    for c in range(n_sr):
        kinds.append(("srbd", (25, 50, 100)[c % 3], c))
    for c in range(n_wb):
        kinds.append(("wb", (50, 100)[c % 2], c))
    for c in range(n_mr):
        kinds.append(("mr", 50, c))
    out = []
    for idx, (kind, N, c) in enumerate(kinds):
        if kind == "srbd":
            model = gen_c2(N, 1000 + c)
        elif kind == "wb":
            model = gen_c1_like(N, 36, 12, [5, 1, c], dt=0.01)
        else:
            model = gen_c4(1000 + c, N=N)
        out.append((model, [5, 2, idx]))
    return out


def x0_walk(model: dict, seed, steps: int, std: float = 1e-2) -> np.ndarray:
    """Initial states of a client's consecutive requests: x0 of the model,
    then x0_{k+1} = x0_k + N(0, std)."""
    rng = np.random.default_rng(seed)
    steps_ = rng.normal(0.0, std, (steps, model["x0"].shape[0]))
    steps_[0] = 0.0
    return model["x0"][None, :] + np.cumsum(steps_, axis=0)


def stack(probs: list) -> dict:
    """List of single-instance dicts -> dict of arrays with a batch axis."""
    return {k: np.stack([p[k] for p in probs]) for k in FIELDS}


def instance(batch: dict, b: int) -> dict:
    return {k: batch[k][b] for k in FIELDS}


def as_dtype(prob: dict, dtype) -> dict:
    return {k: np.ascontiguousarray(v, dtype=dtype) for k, v in prob.items()}


def gen_batch(gen, count: int, dtype=np.float32, workers: int | None = None,
              start: int = 0) -> dict:
    """Draw instances ``start .. start+count-1`` with ``gen(instance)`` into
    contiguous batch-major arrays of ``dtype`` (threads over instances)."""
    first = gen(start)
    shapes = {k: v.shape for k, v in first.items()}
    out = {k: np.empty((count,) + shapes[k], dtype=dtype) for k in FIELDS}

    def fill(i):
        p = first if i == 0 else gen(start + i)
        for k in FIELDS:
            out[k][i] = p[k]

    workers = workers or min(16, os.cpu_count() or 1)
    if count == 1 or workers == 1:
        for i in range(count):
            fill(i)
    else:
        with _cf.ThreadPoolExecutor(workers) as ex:
            list(ex.map(fill, range(count)))
    return out


# ---------------------------------------------------------------------------
# Inputs of the QP-data builder (Gauss-Newton least-squares cost plus relaxed
# barriers): a tracking-like residual eps = [x - x_ref; u - u_ref] whose
# Jacobians are the selection matrices plus N(0, 0.1) perturbations
# (p = n + m rows, so the Gauss-Newton Hessian is positive definite),
# diagonal weights W with the c2 Q/R ranges, and nc linear-in-(x, u)
# constraints with values xi ~ U[-0.05, 1] (about one in seven inside the
# relaxation zone xi < delta = U[0.05, 0.2]) and mu ~ U[0.01, 0.1].  The
# dynamics A, B, c and x0 are drawn as in c1 (dt = 0.02).
QP_FIELDS = ("Ex", "Eu", "e", "W", "Gx", "Gu", "g")


def gen_qpdata(N: int, n: int, m: int, nc: int, seed) -> dict:
    rng = np.random.default_rng(seed)
    p = n + m
    sel_x = np.zeros((p, n))
    sel_x[:n, :n] = np.eye(n)
    sel_u = np.zeros((p, m))
    sel_u[n:, :m] = np.eye(m)
    Ex = sel_x[None] + rng.normal(0.0, 0.1, (N + 1, p, n))
    Eu = sel_u[None] + rng.normal(0.0, 0.1, (N, p, m))
    e = rng.normal(0.0, 0.1, (N + 1, p))
    wd = np.concatenate([rng.uniform(1.0, 100.0, (N + 1, n)), rng.uniform(1e-3, 1e-1, (N + 1, m))], axis=1)
    W = _diag_stack(wd)
    Gx = rng.normal(0.0, 0.1, (N + 1, nc, n))
    Gu = rng.normal(0.0, 1.0, (N, nc, m))
    g = rng.uniform(-0.05, 1.0, (N + 1, nc))
    mu = rng.uniform(0.01, 0.1, nc)
    delta = rng.uniform(0.05, 0.2, nc)
    A = np.eye(n)[None] + 0.02 * rng.normal(0.0, 1.0, (N, n, n))
    B = rng.normal(0.0, 0.1, (N, n, m))
    c = rng.normal(0.0, 1e-3, (N, n))
    x0 = rng.normal(0.0, 0.1, n)
    return {"Ex": Ex, "Eu": Eu, "e": e, "W": W, "Gx": Gx, "Gu": Gu, "g": g, "mu": mu, "delta": delta,
            "A": A, "B": B, "c": c, "x0": x0}


def gen_qp_batch(count: int, N: int, n: int, m: int, nc: int, seed0, dtype=np.float64) -> dict:
    """``count`` instances of gen_qpdata (seeds [seed0..., i]) stacked on a
    batch axis; mu and delta (per constraint, shared by every instance and
    stage) are those of instance 0."""
    insts = [gen_qpdata(N, n, m, nc, list(np.atleast_1d(seed0)) + [i]) for i in range(count)]
    out = {k: np.ascontiguousarray(np.stack([d[k] for d in insts]), dtype=dtype)
           for k in QP_FIELDS + ("A", "B", "c", "x0")}
    out["mu"] = np.ascontiguousarray(insts[0]["mu"], dtype=dtype)
    out["delta"] = np.ascontiguousarray(insts[0]["delta"], dtype=dtype)
    return out


# ---------------------------------------------------------------------------
# Synthetic nonlinear model for the line search and the SQP iteration: the
# c2-like linear part (A = I + dt F, F 30 % nonzero ~ N(0, 1); B ~ N(0, dt);
# c ~ N(0, 1e-3)) plus a bilinear term gamma (P x) * (V u) with P, V ~
# N(0, 1/sqrt(n)), gamma = `gamma`; tracking references xr ~ N(0, 0.1),
# ur = 0, weights wx ~ U[1, 10], wu ~ U[0.01, 0.1]; nc linear constraints
# Gx ~ N(0, 0.1), Gu ~ N(0, 1), g0 ~ U[0.2, 1] (feasible at x = u = 0) with
# barrier parameters mu ~ U[0.01, 0.1], delta ~ U[0.05, 0.2]; the measured
# initial state xhat0 ~ N(0, 0.5).
MODEL_FIELDS = ("A", "B", "c", "P", "V", "xr", "ur", "wx", "wu", "Gx", "Gu", "g0")


def gen_bilinear(N: int, n: int, m: int, nc: int, seed, gamma: float = 0.05, dt: float = 0.02) -> dict:
    rng = np.random.default_rng(seed)
    A = np.eye(n) + dt * _sparse(rng, (n, n), 0.3, 1.0)
    B = rng.normal(0.0, dt, (n, m))
    c = rng.normal(0.0, 1e-3, n)
    P = rng.normal(0.0, 1.0 / np.sqrt(n), (n, n))
    V = rng.normal(0.0, 1.0 / np.sqrt(n), (n, m))
    xr = rng.normal(0.0, 0.1, (N + 1, n))
    ur = np.zeros((N, m))
    wx = rng.uniform(1.0, 10.0, (N + 1, n))
    wu = rng.uniform(0.01, 0.1, (N, m))
    Gx = rng.normal(0.0, 0.1, (nc, n))
    Gu = rng.normal(0.0, 1.0, (nc, m))
    g0 = rng.uniform(0.2, 1.0, nc)
    mu = rng.uniform(0.01, 0.1, nc)
    delta = rng.uniform(0.05, 0.2, nc)
    xhat0 = rng.normal(0.0, 0.5, n)
    return {"A": A, "B": B, "c": c, "P": P, "V": V, "gamma": float(gamma), "xr": xr, "ur": ur, "wx": wx, "wu": wu,
            "Gx": Gx, "Gu": Gu, "g0": g0, "mu": mu, "delta": delta, "xhat0": xhat0}


def gen_bilinear_batch(count: int, N: int, n: int, m: int, nc: int, seed0, gamma: float = 0.05,
                       dtype=np.float64) -> dict:
    """``count`` models of gen_bilinear (seeds [seed0..., i]) with a batch
    axis on every array; gamma, mu and delta are shared (instance 0's)."""
    ms = [gen_bilinear(N, n, m, nc, list(np.atleast_1d(seed0)) + [i], gamma) for i in range(count)]
    out = {k: np.ascontiguousarray(np.stack([d[k] for d in ms]), dtype=dtype) for k in MODEL_FIELDS + ("xhat0",)}
    out["mu"] = np.ascontiguousarray(ms[0]["mu"], dtype=dtype)
    out["delta"] = np.ascontiguousarray(ms[0]["delta"], dtype=dtype)
    out["gamma"] = float(gamma)
    return out


def model_instance(batch: dict, b: int) -> dict:
    """One model of a gen_bilinear_batch dict."""
    d = {k: batch[k][b] for k in MODEL_FIELDS + ("xhat0",)}
    d.update(gamma=batch["gamma"], mu=batch["mu"], delta=batch["delta"])
    return d
