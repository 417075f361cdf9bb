"""The one-launch solve (mapping fused = 2): one workgroup of several
wavefronts per instance runs the elements, the reverse scan, the policy, the
forward scan, the recovery, the FP64 residual and the refinement sweeps in
a single kernel, through the C ABI.

It runs the task bodies of the launch sequence in the same phase order, so
its FP32 outputs (solution, residual, status) must equal the launched
form's bit for bit; FP64 solves meet the 1e-9 bar against the oracle.  An
instance flagged for the FP64 fallback is recomputed whole with FP64
arithmetic by a second launch; the others keep the FP32 bits."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import oracle_check, run, say, to_dev

pytestmark = pytest.mark.gpu

# (N, n, m): every wavefront class (orders 4, 12, 20, 36, 64), N = 1, m > n,
# ragged trees
SHAPES = [(1, 4, 2), (16, 4, 2), (25, 12, 12), (13, 8, 3), (7, 20, 9), (33, 36, 12), (6, 64, 64), (5, 3, 17)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401  (raises if the library is missing)


def _pin(batch, N, n, m, fused, dtypes=None):
    import torch
    import paper_2506_07823_amd as L
    for dt in dtypes or (torch.float32, torch.float64):
        if fused is None:
            L.set_tuning(batch, N, n, m, dt, clear=True)
        else:
            L.set_tuning(batch, N, n, m, dt, engine="wavefront", fused=fused)


def _runs(b, dt, forms, **kw):
    N, n, m = b["B"].shape[1:]
    count = b["A"].shape[0]
    outs = []
    try:
        for f in forms:
            _pin(count, N, n, m, f)
            outs.append(run(b, dt, **kw))
    finally:
        _pin(count, N, n, m, None)
    return outs


@pytest.mark.parametrize("N,n,m", SHAPES)
def test_fused_fp64_meets_oracle(N, n, m):
    b = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[900, N, n, m, i]), 3, np.float64)
    say(f"[fused fp64] N={N} n={n} m={m} batch=3")
    (out,) = _runs(b, np.float64, [2], want_resid=True)
    assert not out["status"].any(), out["status"]
    for i in range(3):
        errs, res = oracle_check(b, out, i)
        say(f"  inst {i}: rel err {errs}, oracle resid {res:.2e}, gpu resid {out['resid'][i]:.2e}")
        assert max(errs) <= 1e-9 and res <= 1e-11, (i, errs)


@pytest.mark.parametrize("N,n,m", SHAPES)
def test_fused_fp32_bitwise_equals_launched(N, n, m):
    b = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[910, N, n, m, i]), 3, np.float32)
    say(f"[fused fp32 vs launched] N={N} n={n} m={m} batch=3")
    per_inst, fused = _runs(b, np.float32, [1, 2], refine=2, want_resid=True)
    for f in ("x", "u", "lam", "status", "resid"):
        assert np.array_equal(per_inst[f], fused[f]), f
    assert fused["resid"].max() <= 1e-5


def test_fused_srbd_batch_residual():
    """SRBD-shaped horizon N = 100, batch 64: every residual meets the bar
    and sampled instances match the oracle."""
    b = synth.gen_batch(lambda i: synth.gen_c2(100, i), 64, np.float32)
    say("[fused srbd] N=100 n=m=12 batch=64")
    (out,) = _runs(b, np.float32, [2], want_resid=True)
    assert not out["status"].any()
    say(f"  max gpu resid {out['resid'].max():.2e}")
    assert out["resid"].max() <= 1e-5
    for i in (0, 63):
        errs, res = oracle_check(b, out, i, as_f32=True)
        assert res <= 1e-5 and max(errs) <= 1e-3, (i, errs, res)


def test_fused_fallback_redoes_only_flagged_instance():
    b = synth.gen_batch(lambda i: synth.gen_c1_like(12, 8, 4, [920, i]), 3, np.float32)
    b["R"][2, 5] = np.diag([1e-7, 1.0, 1.0, 1.0])
    say("[fused fallback] cond(R) = 1e7 in instance 2")
    per_inst, fused = _runs(b, np.float32, [1, 2], want_resid=True, refine=4)
    assert fused["status"][2] == 8, fused["status"]
    assert fused["status"][0] == 0 and fused["status"][1] == 0
    for f in ("x", "u", "lam", "resid"):
        assert np.array_equal(per_inst[f][:2], fused[f][:2]), f
    errs, res = oracle_check(b, fused, 2, as_f32=True)
    say(f"  fallback instance: rel err {errs}, resid gpu {fused['resid'][2]:.2e} oracle {res:.2e}")
    assert fused["resid"][2] <= 1e-5 and res <= 1e-5


def test_fused_indefinite_R_flags_only_that_instance():
    b = synth.gen_batch(lambda i: synth.gen_rand(10, 6, 3, seed=[930, i]), 3, np.float32)
    b["R"][1, 4] = -100.0 * np.eye(3)
    say("[fused status indefinite R]")
    (out,) = _runs(b, np.float32, [2])
    assert out["status"][1] & 2
    assert out["status"][0] == 0 and out["status"][2] == 0


def test_fused_warm_start_equals_launched():
    import torch
    import paper_2506_07823_amd as L
    N, n, m = 20, 12, 12
    b = synth.gen_batch(lambda i: synth.gen_c2(N, i), 4, np.float32)
    dev = to_dev(b, np.float32)
    args = [dev[k] for k in L.FIELDS]
    cold = L.solve(*args)
    torch.cuda.synchronize()
    g = torch.Generator(device="cpu").manual_seed(931)
    warm = tuple((cold[f] + 1e-3 * torch.randn(cold[f].shape, generator=g).to(cold[f])).contiguous()
                 for f in ("x", "u", "lam"))
    say("[fused warm start] N=20 n=m=12 batch=4")
    outs = []
    try:
        for fused in (1, 2):
            _pin(4, N, n, m, fused, (torch.float32,))
            o = L.solve(*args, warm=warm, refine=2, want_resid=True)
            torch.cuda.synchronize()
            outs.append({k: v.cpu().numpy() for k, v in o.items()})
    finally:
        _pin(4, N, n, m, None, (torch.float32,))
    for f in ("x", "u", "lam", "status", "resid"):
        assert np.array_equal(outs[0][f], outs[1][f]), f
    assert outs[1]["resid"].max() <= 1e-5


def test_fused_graph_replay_matches_eager():
    import torch
    import paper_2506_07823_amd as L
    N, n, m = 50, 12, 12
    batch = synth.gen_batch(lambda i: synth.gen_c2(N, i), 4, np.float32)
    say("[fused graph replay] N=50 n=m=12 batch=4")
    dev = to_dev(batch, np.float32)
    args = [dev[k] for k in L.FIELDS]
    _pin(4, N, n, m, 2, (torch.float32,))
    try:
        eager = L.solve(*args, want_resid=True)
        torch.cuda.synchronize()
        ref = {k: v.clone() for k, v in eager.items()}
        ws = L.Workspace()
        out = L.solve(*args, want_resid=True, workspace=ws)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            L.solve(*args, want_resid=True, workspace=ws, out=out)
        torch.cuda.synchronize()
        for rep in range(4):
            for v in out.values():
                v.fill_(-1)
            ws.buf.fill_(0x7f)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for k in ("x", "u", "lam", "status", "resid"):
                assert torch.equal(out[k], ref[k]), (rep, k)
    finally:
        _pin(4, N, n, m, None, (torch.float32,))
