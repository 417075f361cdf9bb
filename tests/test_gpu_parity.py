"""GPU parity of the HIP path against the CPU FP64 oracle, through the C ABI.

Tolerances: the FP64 paths (scan and sequential Riccati) must reach relative
error <= 1e-9 per output block; the FP32 scan with one FP64-residual
refinement sweep must reach a relative KKT residual <= 1e-5 (measured both
on the GPU and, independently, by the oracle on the returned solution), and
its relative error against the oracle (solved on the same FP32-rounded
inputs) is reported and bounded loosely (it is limited by FP32 storage of
the result times the conditioning of the instance).
"""
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


@pytest.mark.parametrize("method", ["scan", "plain"])
def test_tiny_case_fp64(method):
    batch = synth.gen_batch(synth.gen_c1, 3, np.float64)
    say(f"[tiny fp64 {method}] N=16 n=4 m=2 batch=3")
    out = run(batch, np.float64, method=method, want_resid=True)
    assert not out["status"].any(), out["status"]
    for b in range(3):
        errs, res = oracle_check(batch, out, b)
        say(f"  inst {b}: rel err x/u/lam = {errs}, oracle resid {res:.2e}, gpu resid {out['resid'][b]:.2e}")
        assert max(errs) <= FP64_TOL
        assert res <= 1e-12 and out["resid"][b] <= 1e-12


# (N, n, m): every padded-order class (max(n, m) up to 8/16/24/32/40/48/64),
# horizons with ragged tree levels, N = 1 and N = 2, m > n and m = n.
SHAPES = [(1, 1, 1), (2, 3, 1), (5, 4, 4), (7, 3, 2), (16, 4, 2), (13, 8, 3), (33, 12, 12),
          (9, 17, 5), (10, 20, 9), (8, 30, 30), (20, 36, 12), (6, 40, 7), (11, 45, 20), (3, 64, 64),
          (4, 5, 9)]


@pytest.mark.parametrize("N,n,m", SHAPES)
@pytest.mark.parametrize("method", ["scan", "plain"])
def test_shapes_fp64(N, n, m, method):
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[200, N, n, m, i]), 3, np.float64)
    say(f"[shapes fp64 {method}] N={N} n={n} m={m} batch=3")
    out = run(batch, np.float64, method=method)
    assert not out["status"].any(), out["status"]
    for b in range(3):
        errs, res = oracle_check(batch, out, b)
        assert max(errs) <= FP64_TOL, (b, errs)
        assert res <= 1e-11


@pytest.mark.parametrize("N", synth.C2_HORIZONS)
def test_srbd_shaped_fp32_refined(N):
    batch = synth.gen_batch(lambda i: synth.gen_c2(N, i), 2, np.float32)
    say(f"[srbd fp32 refined] N={N} n=m=12 batch=2")
    out = run(batch, np.float32, want_resid=True)
    raw = run(batch, np.float32, refine=0, want_resid=True)
    assert not out["status"].any(), out["status"]
    for b in range(2):
        errs, res = oracle_check(batch, out, b, as_f32=True)
        say(f"  inst {b}: rel err {errs}, resid gpu {out['resid'][b]:.2e} oracle {res:.2e} "
            f"(unrefined {raw['resid'][b]:.2e})")
        assert out["resid"][b] <= RESID_TOL and res <= RESID_TOL
        assert max(errs) <= FP32_ERR_BOUND
        assert out["resid"][b] <= raw["resid"][b]


@pytest.mark.parametrize("N,n,m", [(7, 3, 2), (20, 36, 12), (33, 12, 12), (5, 40, 7)])
def test_shapes_fp32_refined(N, n, m):
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[300, N, n, m, i]), 3, np.float32)
    say(f"[shapes fp32 refined] N={N} n={n} m={m}")
    out = run(batch, np.float32, want_resid=True)
    assert not out["status"].any(), out["status"]
    for b in range(3):
        errs, res = oracle_check(batch, out, b, as_f32=True)
        assert out["resid"][b] <= RESID_TOL and res <= RESID_TOL, (b, out["resid"][b], res)
        assert max(errs) <= FP32_ERR_BOUND, errs


def test_whole_body_full_batch():
    """n=36, m=12, N=100, batch 4096 in the benchmark's launch configuration:
    every instance's GPU residual, plus sampled instances against the oracle."""
    batch = synth.gen_batch(synth.gen_c3, 4096, np.float32)
    say("[whole-body fp32 refined] N=100 n=36 m=12 batch=4096")
    out = run(batch, np.float32, want_resid=True)
    assert not out["status"].any()
    say(f"  max gpu resid {out['resid'].max():.2e}")
    assert out["resid"].max() <= RESID_TOL
    for b in (0, 1, 777, 2048, 4095):
        errs, res = oracle_check(batch, out, b, as_f32=True)
        say(f"  inst {b}: rel err {errs}, oracle resid {res:.2e}")
        assert res <= RESID_TOL and max(errs) <= FP32_ERR_BOUND


def test_whole_body_plain_fp64_sample():
    batch = synth.gen_batch(synth.gen_c3, 64, np.float64)
    say("[whole-body plain fp64] N=100 n=36 m=12 batch=64")
    out = run(batch, np.float64, method="plain", want_resid=True)
    assert not out["status"].any()
    for b in (0, 31, 63):
        errs, res = oracle_check(batch, out, b)
        assert max(errs) <= FP64_TOL and res <= 1e-11


def test_alone_equals_in_batch():
    """Per-instance arithmetic does not depend on the batch it is solved in."""
    batch = synth.gen_batch(synth.gen_c3, 8, np.float32)
    say("[alone vs batch] n=36 batch=8")
    full = run(batch, np.float32)
    for b in (0, 5):
        one = {k: v[b:b + 1] for k, v in batch.items()}
        alone = run(one, np.float32)
        for f in ("x", "u", "lam"):
            assert np.array_equal(alone[f][0], full[f][b])


def test_deterministic():
    batch = synth.gen_batch(lambda i: synth.gen_c2(50, i), 4, np.float32)
    say("[determinism] srbd N=50 batch=4")
    a = run(batch, np.float32)
    b = run(batch, np.float32)
    for f in ("x", "u", "lam"):
        assert np.array_equal(a[f], b[f])


def test_per_instance_path_fp64_and_matches_level_path():
    """The per-instance form of the vector-only passes (one workgroup walks
    an instance; pinned here as the mapping of a batch of 160) calls the same
    task bodies in the same order as the level-by-level launches, so an
    instance solved in that batch equals the same instance solved alone
    (level by level), bit for bit."""
    import torch
    import paper_2506_07823_amd as L
    batch = synth.gen_batch(lambda i: synth.gen_rand(13, 8, 3, seed=[500, i]), 160, np.float64)
    say("[per-instance path fp64] N=13 n=8 m=3 batch=160")
    L.set_tuning(160, 13, 8, 3, torch.float64, fused=True)
    L.set_tuning(160, 13, 8, 3, torch.float32, fused=True)
    try:
        out = run(batch, np.float64, want_resid=True)
        b32 = {k: v.astype(np.float32) for k, v in batch.items()}
        full = run(b32, np.float32, refine=2, want_resid=True)
    finally:
        L.set_tuning(160, 13, 8, 3, torch.float64, clear=True)
        L.set_tuning(160, 13, 8, 3, torch.float32, clear=True)
    assert not out["status"].any()
    for b in (0, 77, 159):
        errs, res = oracle_check(batch, out, b)
        assert max(errs) <= FP64_TOL and res <= 1e-11
    for b in (3, 150):
        alone = run({k: v[b:b + 1] for k, v in b32.items()}, np.float32, refine=2, want_resid=True)
        for f in ("x", "u", "lam", "resid"):
            assert np.array_equal(alone[f][0], full[f][b]), f
