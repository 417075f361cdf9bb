"""Split schedule of the reverse scan (mapping split = 1, wavefront engine):
the balanced tree covers the first 2^k scan elements (the largest power of
two below N + 1) and a sequential sweep of combines with the complete suffix
to their right covers the rest, through the C ABI.

The value functions are the same in exact arithmetic, so FP64 solves meet
the 1e-9 bar against the oracle and FP32 solves meet the residual bar after
refinement; the FP64 fallback of a flagged sweep redoes that instance's
whole sweep."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import oracle_check, run, say, to_dev

pytestmark = pytest.mark.gpu

# (N, n, m) with the head size 2^k and the sweep length N - 2^k:
# N=1 (head 1, sweep 0), N=2 (2, 0), N=16 (16, 0), N=13 (8, 5), N=25 (16, 9),
# N=33 (32, 1), N=100 (64, 36), m > n, order 64
SHAPES = [(1, 4, 2), (2, 4, 2), (16, 4, 2), (13, 8, 3), (25, 12, 12), (33, 36, 12), (100, 36, 12), (5, 3, 17),
          (6, 64, 64)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401  (raises if the library is missing)


def _pinned(batch, N, n, m, dtype, split, fused=0, **kw):
    import torch
    import paper_2506_07823_amd as L
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    count = batch["A"].shape[0]
    L.set_tuning(count, N, n, m, tdt, engine="wavefront", fused=fused, split=split)
    try:
        return run(batch, dtype, **kw)
    finally:
        L.set_tuning(count, N, n, m, tdt, clear=True)


@pytest.mark.parametrize("N,n,m", SHAPES)
def test_split_fp64_meets_oracle(N, n, m):
    b = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[950, N, n, m, i]), 3, np.float64)
    say(f"[split fp64] N={N} n={n} m={m} batch=3")
    out = _pinned(b, N, n, m, np.float64, True, want_resid=True)
    assert not out["status"].any(), out["status"]
    for i in range(3):
        errs, res = oracle_check(b, out, i)
        assert max(errs) <= 1e-9 and res <= 1e-11, (i, errs, res)


@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("N,n,m", [(25, 12, 12), (100, 36, 12), (13, 8, 3)])
def test_split_fp32_meets_residual(N, n, m, fused):
    b = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[951, N, n, m, i]), 4, np.float32)
    say(f"[split fp32] N={N} n={n} m={m} fused={fused} batch=4")
    out = _pinned(b, N, n, m, np.float32, True, fused=fused, want_resid=True, refine=4)
    assert not out["status"].any(), out["status"]
    assert out["resid"].max() <= 1e-5, out["resid"]
    for i in range(4):
        errs, res = oracle_check(b, out, i, as_f32=True)
        assert res <= 1e-5 and max(errs) <= 1e-3, (i, errs, res)


def test_split_whole_body_full_batch_sampled():
    """The whole-body workload (n = 36, m = 12, N = 100) at its full batch of
    4096 with the split schedule pinned: every instance meets the residual
    bar (library FP64 residual, refinement as in the benchmark), sampled
    instances also against the oracle."""
    N, n, m, count = 100, 36, 12, 4096
    b = synth.gen_batch(synth.gen_c3, count, np.float32)
    say(f"[split whole-body] batch={count}")
    out = _pinned(b, N, n, m, np.float32, True, want_resid=True, refine=2)
    assert not out["status"].any()
    assert out["resid"].max() <= 1e-5, float(out["resid"].max())
    for i in (0, 1, 2047, 4095):
        errs, res = oracle_check(b, out, i, as_f32=True)
        say(f"  instance {i}: rel err {errs}, oracle resid {res:.2e}")
        assert res <= 1e-5 and max(errs) <= 1e-3, (i, errs, res)


def test_split_sweep_fallback_redoes_the_instance():
    """A terminal weight with condition 3.3e6 flags the first combine of the
    sequential sweep (its P2 is Q_N): the instance's sweep is redone in FP64
    (status bit 8 only), the others keep clean status words, and the
    tolerance is met as on the balanced tree."""
    N, n, m = 25, 12, 12
    b = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[952, i]), 3, np.float32)
    b["Q"][1, N] = np.diag([3e-3] + [1.0] * (n - 2) + [1e4])
    say("[split sweep fallback]")
    out = _pinned(b, N, n, m, np.float32, True, want_resid=True, refine=4)
    ref = _pinned(b, N, n, m, np.float32, False, want_resid=True, refine=4)
    assert out["status"][1] == 8, out["status"]
    assert out["status"][0] == 0 and out["status"][2] == 0, out["status"]
    assert ref["status"][1] == 8, ref["status"]
    errs, res = oracle_check(b, out, 1, as_f32=True)
    say(f"  flagged instance: rel err {errs}, resid gpu {out['resid'][1]:.2e} oracle {res:.2e}")
    assert out["resid"][1] <= 1e-5 and res <= 1e-5


def test_split_in_a_graph_replays_identically():
    """Captured into a HIP graph, replays of the split schedule give the
    bits of the eager solve, with the outputs and the whole workspace
    overwritten between replays (nothing reads a record the solve did not
    write)."""
    import torch
    import paper_2506_07823_amd as L
    N, n, m, count = 25, 12, 12, 8
    b = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[953, i]), count, np.float32)
    dev = to_dev(b, np.float32)
    args = [dev[k] for k in L.FIELDS]
    L.set_tuning(count, N, n, m, torch.float32, engine="wavefront", fused=0, split=True)
    try:
        eager = L.solve(*args, want_resid=True)
        torch.cuda.synchronize()
        ref = {k: v.clone() for k, v in eager.items()}
        ws = L.Workspace()
        out = L.solve(*args, want_resid=True, workspace=ws)      # sizes the workspace
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            L.solve(*args, want_resid=True, workspace=ws, out=out)
        torch.cuda.synchronize()
        for rep in range(3):
            for v in out.values():
                v.fill_(-1)
            ws.buf.fill_(0x7f)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for k in ("x", "u", "lam", "status", "resid"):
                assert torch.equal(out[k], ref[k]), (rep, k)
    finally:
        L.set_tuning(count, N, n, m, torch.float32, clear=True)


def test_split_rejected_off_the_wavefront_engine():
    import torch
    import paper_2506_07823_amd as L
    with pytest.raises(Exception):
        L.set_tuning(4, 10, 80, 12, torch.float32, engine="matrix-core", split=True)
    with pytest.raises(Exception):
        L.set_tuning(4, 10, 12, 12, torch.float32, engine="wavefront", fused=2, split=True)
