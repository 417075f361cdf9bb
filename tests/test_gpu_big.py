"""GPU parity of the large-block engine (orders 65..256: one workgroup per
task, products on matrix cores) against the CPU FP64 oracle, through the C ABI.

Same bars as the small-block classes: FP64 scan and plain paths within 1e-9
relative error per output block; FP32 scan with FP64-residual refinement at a
relative KKT residual <= 1e-5 (GPU and oracle residual of the returned
solution)."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import oracle_check, run, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9
RESID_TOL = 1e-5
FP32_ERR_BOUND = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401  (raises if the library is missing)


# (N, n, m): just above the wavefront engine's limit, ragged 64-tiles and
# 32-blocks, m > n, m = n, N = 1, a ragged tree, and the largest order.
BIG_SHAPES = [(5, 65, 3), (7, 80, 70), (4, 100, 130), (1, 70, 70), (33, 72, 24), (6, 130, 40), (3, 192, 192),
              (2, 256, 17)]


@pytest.mark.parametrize("N,n,m", BIG_SHAPES)
@pytest.mark.parametrize("method", ["scan", "plain"])
def test_big_shapes_fp64(N, n, m, method):
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[600, N, n, m, i]), 2, np.float64)
    say(f"[big fp64 {method}] N={N} n={n} m={m} batch=2")
    out = run(batch, np.float64, method=method)
    assert not out["status"].any(), out["status"]
    for b in range(2):
        errs, res = oracle_check(batch, out, b)
        say(f"  inst {b}: rel err x/u/lam = {errs}, oracle resid {res:.2e}")
        assert max(errs) <= FP64_TOL, (b, errs)
        assert res <= 1e-11


@pytest.mark.parametrize("N,n,m", [(7, 80, 40), (9, 130, 40), (4, 192, 192)])
def test_big_shapes_fp32_refined(N, n, m):
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[610, N, n, m, i]), 2, np.float32)
    say(f"[big fp32 refined] N={N} n={n} m={m}")
    out = run(batch, np.float32, want_resid=True)
    assert not out["status"].any(), out["status"]
    for b in range(2):
        errs, res = oracle_check(batch, out, b, as_f32=True)
        say(f"  inst {b}: rel err {errs}, resid gpu {out['resid'][b]:.2e} oracle {res:.2e}")
        assert out["resid"][b] <= RESID_TOL and res <= RESID_TOL
        assert max(errs) <= FP32_ERR_BOUND


def test_multi_robot_full_batch():
    """n = m = 192 (16 coupled SRBD-like robots), N = 50, batch 64: every
    instance's GPU residual, sampled instances against the oracle."""
    batch = synth.gen_batch(synth.gen_c4, 64, np.float32)
    say("[multi-robot fp32 refined] N=50 n=m=192 batch=64")
    out = run(batch, np.float32, want_resid=True)
    assert not out["status"].any(), out["status"]
    say(f"  max gpu resid {out['resid'].max():.2e}")
    assert out["resid"].max() <= RESID_TOL
    for b in (0, 63):
        errs, res = oracle_check(batch, out, b, as_f32=True)
        say(f"  inst {b}: rel err {errs}, oracle resid {res:.2e}")
        assert res <= RESID_TOL and max(errs) <= FP32_ERR_BOUND


def test_multi_robot_plain_fp64_sample():
    batch = synth.gen_batch(synth.gen_c4, 2, np.float64)
    say("[multi-robot plain fp64] N=50 n=m=192 batch=2")
    out = run(batch, np.float64, method="plain", want_resid=True)
    assert not out["status"].any()
    errs, res = oracle_check(batch, out, 1)
    say(f"  inst 1: rel err {errs}, oracle resid {res:.2e}")
    assert max(errs) <= FP64_TOL and res <= 1e-11


def test_big_alone_equals_in_batch():
    batch = synth.gen_batch(lambda i: synth.gen_rand(6, 90, 30, seed=[620, i]), 5, np.float32)
    say("[big alone vs batch] N=6 n=90 m=30 batch=5")
    full = run(batch, np.float32, want_resid=True)
    for b in (0, 4):
        alone = run({k: v[b:b + 1] for k, v in batch.items()}, np.float32, want_resid=True)
        for f in ("x", "u", "lam", "resid"):
            assert np.array_equal(alone[f][0], full[f][b]), f


def test_big_per_instance_path():
    """The per-instance form of the vector-only passes (pinned for this
    batch of 130): same bits as the level-by-level launches of an alone
    solve."""
    import torch
    import paper_2506_07823_amd as L
    batch = synth.gen_batch(lambda i: synth.gen_rand(5, 66, 8, seed=[630, i]), 130, np.float64)
    say("[big per-instance path fp64] N=5 n=66 m=8 batch=130")
    for dt in (torch.float64, torch.float32):
        L.set_tuning(130, 5, 66, 8, dt, fused=True)
    try:
        out = run(batch, np.float64, want_resid=True)
        b32 = {k: v.astype(np.float32) for k, v in batch.items()}
        full = run(b32, np.float32, refine=2, want_resid=True)
    finally:
        for dt in (torch.float64, torch.float32):
            L.set_tuning(130, 5, 66, 8, dt, clear=True)
    assert not out["status"].any()
    for b in (0, 129):
        errs, res = oracle_check(batch, out, b)
        assert max(errs) <= FP64_TOL and res <= 1e-11
    alone = run({k: v[7:8] for k, v in b32.items()}, np.float32, refine=2, want_resid=True)
    for f in ("x", "u", "lam", "resid"):
        assert np.array_equal(alone[f][0], full[f][7]), f


@pytest.mark.parametrize("method", ["scan", "plain"])
def test_big_indefinite_R_flags_only_that_instance(method):
    dt = np.float64 if method == "plain" else np.float32
    b = synth.gen_batch(lambda i: synth.gen_rand(6, 70, 12, seed=[640, i]), 3, dt)
    b["R"][1, 2] = -100.0 * np.eye(12)
    say(f"[big status indefinite R {method}]")
    out = run(b, dt, method=method)
    assert out["status"][1] & 2
    assert out["status"][0] == 0 and out["status"][2] == 0
