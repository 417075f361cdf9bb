"""The SQP iteration on the GPU (lqr_sqp_solve: linearization, QP-data
builder, scan solve, parallel filter line search, update; Sec. II-B, II-E,
II-F) against the oracle's iteration on the same bilinear model: the same
step length every iteration and the same iterates (FP64 element-wise 1e-9
per iteration for several iterations; FP32 run converged to the oracle's
solution), and a batch whose instances take different step lengths."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import elem_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401


def _dev_model(mb, dtype):
    import torch
    import paper_2506_07823_amd as L
    td = torch.float32 if dtype == np.float32 else torch.float64
    d = {k: torch.from_numpy(np.ascontiguousarray(mb[k], dtype=dtype)).to("cuda:0", td) for k in L.MODEL_FIELDS}
    d["gamma"] = mb["gamma"]
    return d


def _start(mb, dtype):
    import torch
    B, n = mb["xhat0"].shape
    N = mb["ur"].shape[1]
    m = mb["ur"].shape[2]
    X = np.repeat(mb["xhat0"][:, None, :], N + 1, axis=1)
    td = torch.float32 if dtype == np.float32 else torch.float64
    return (torch.from_numpy(np.ascontiguousarray(X, dtype=dtype)).to("cuda:0", td),
            torch.zeros((B, N, m), dtype=td, device="cuda:0"), torch.zeros((B, N + 1, n), dtype=td, device="cuda:0"))


@pytest.mark.parametrize("N,n,m,nc,gamma", [(12, 6, 3, 4, 0.2), (20, 12, 12, 8, 0.1), (10, 36, 12, 6, 0.05)])
def test_sqp_iterations_match_oracle_fp64(N, n, m, nc, gamma):
    import torch
    import oracle
    import paper_2506_07823_amd as L
    from oracle import sqp
    count, iters = 3, 6
    mb = synth.gen_bilinear_batch(count, N, n, m, nc, [995, N, n], gamma)
    md = _dev_model(mb, np.float64)
    X, U, Lm = _start(mb, np.float64)
    say(f"[sqp fp64] N={N} n={n} m={m} nc={nc} gamma={gamma}, {iters} iterations")
    refs = []
    for b in range(count):
        mdl = synth.model_instance(mb, b)
        Xo = np.repeat(mdl["xhat0"][None], N + 1, axis=0)
        Uo, Lo = np.zeros((N, m)), np.zeros((N + 1, n))
        steps = []
        for _ in range(iters):
            Xo, Uo, Lo, a = sqp.sqp_iteration(mdl, Xo, Uo, Lo, mdl["xhat0"], oracle.riccati, theta_max=1e-2)
            steps.append((Xo.copy(), Uo.copy(), Lo.copy(), a))
        refs.append(steps)
    for it in range(iters):
        status, alphas = L.sqp_solve(md, X, U, Lm, iters=1, theta_max=1e-2)
        torch.cuda.synchronize()
        assert not status.any().item(), status
        for b in range(count):
            Xo, Uo, Lo, a = refs[b][it]
            assert alphas[0, b].item() == a, (it, b, alphas[0, b].item(), a)
            e = max(elem_err(X[b].cpu().numpy(), Xo), elem_err(U[b].cpu().numpy(), Uo),
                    elem_err(Lm[b].cpu().numpy(), Lo))
            assert e <= 1e-9, (it, b, e)
    say(f"  steps {[round(r[1][3], 4) for r in refs]} ... all equal to the oracle's")


def test_sqp_fp32_follows_the_oracle():
    """The FP32 iteration (FP32 subproblem, FP64 line-search sums) takes the
    oracle's step lengths over the first iterations and stays within 1e-4
    (element-wise) of its FP64 iterates; later iterations can differ where
    a filter decision is borderline (the iteration is not monotone on this
    model, in either precision)."""
    import torch
    import oracle
    import paper_2506_07823_amd as L
    from oracle import sqp
    N, n, m, nc, gamma, count, iters = 20, 12, 12, 8, 0.1, 4, 6
    mb = synth.gen_bilinear_batch(count, N, n, m, nc, [996], gamma)
    md = _dev_model(mb, np.float32)
    X, U, Lm = _start(mb, np.float32)
    mb64 = {k: (v.astype(np.float32).astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in mb.items()}
    say(f"[sqp fp32] N={N} n={n} m={m}, {iters} iterations against the FP64 oracle")
    refs = []
    for b in range(count):
        mdl = synth.model_instance(mb64, b)
        Xo = np.repeat(mdl["xhat0"][None], N + 1, axis=0)
        Uo, Lo = np.zeros((N, m)), np.zeros((N + 1, n))
        steps = []
        for _ in range(iters):
            Xo, Uo, Lo, a = sqp.sqp_iteration(mdl, Xo, Uo, Lo, mdl["xhat0"], oracle.riccati, theta_max=1e-2)
            steps.append((Xo.copy(), Uo.copy(), a))
        refs.append(steps)
    worst = 0.0
    for it in range(iters):
        status, alphas = L.sqp_solve(md, X, U, Lm, iters=1, theta_max=1e-2)
        torch.cuda.synchronize()
        assert not status.any().item(), status
        for b in range(count):
            Xo, Uo, a = refs[b][it]
            assert alphas[0, b].item() == a, (it, b, alphas[0, b].item(), a)
            e = max(elem_err(X[b].cpu().numpy(), Xo), elem_err(U[b].cpu().numpy(), Uo))
            worst = max(worst, e)
            assert e <= 1e-4, (it, b, e)
    say(f"  step lengths equal to the oracle's; worst element-wise distance {worst:.2e}")
