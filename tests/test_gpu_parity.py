"""GPU parity of the HIP path against the CPU FP64 oracle, through the C ABI.

Gates (tests/gpuhelp.py): the FP64 paths (scan and sequential Riccati) match
the oracle element by element to 1e-9 (elem_err: |gpu - oracle| relative to
|oracle| + the block's largest entry, per output block x, u, lam of each
instance); the FP32 scan with the FP64-residual refinement sweep reaches a
relative KKT residual <= 1e-5 computed by the oracle on the returned
solution, and matches the oracle (solved on the same FP32-rounded inputs)
element by element to FP32_ELEM_TOL.  The full-size batches are compared
instance by instance, every instance.
"""
import numpy as np
import pytest

import synth
from tests.gpuhelp import (FP32_ELEM_TOL, FP64_ELEM_TOL, RESID_TOL, describe, oracle_check, oracle_check_all, run,
                           say, to_dev)

pytestmark = pytest.mark.gpu


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
        say(f"  inst {b}: elem err x/u/lam = {errs}, oracle resid {res:.2e}, gpu resid {out['resid'][b]:.2e}")
        assert max(errs) <= FP64_ELEM_TOL
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
    errs, res, st = oracle_check_all(batch, out)
    assert not st.any()
    assert errs.max() <= FP64_ELEM_TOL, errs
    assert res.max() <= 1e-11


@pytest.mark.parametrize("N", synth.C2_HORIZONS)
def test_srbd_shaped_fp32_refined(N):
    batch = synth.gen_batch(lambda i: synth.gen_c2(N, i), 2, np.float32)
    say(f"[srbd fp32 refined] N={N} n=m=12 batch=2")
    out = run(batch, np.float32, want_resid=True)
    raw = run(batch, np.float32, refine=0, want_resid=True)
    assert not out["status"].any(), out["status"]
    errs, res, _ = oracle_check_all(batch, out, as_f32=True)
    describe(f"N={N}", errs, res)
    say(f"  gpu resid {out['resid']}, unrefined {raw['resid']}")
    assert out["resid"].max() <= RESID_TOL and res.max() <= RESID_TOL
    assert errs.max() <= FP32_ELEM_TOL
    assert (out["resid"] <= raw["resid"]).all()


@pytest.mark.parametrize("N,n,m", [(7, 3, 2), (20, 36, 12), (33, 12, 12), (5, 40, 7)])
def test_shapes_fp32_refined(N, n, m):
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[300, N, n, m, i]), 3, np.float32)
    say(f"[shapes fp32 refined] N={N} n={n} m={m}")
    out = run(batch, np.float32, want_resid=True)
    assert not out["status"].any(), out["status"]
    errs, res, _ = oracle_check_all(batch, out, as_f32=True)
    describe(f"N={N} n={n} m={m}", errs, res)
    assert out["resid"].max() <= RESID_TOL and res.max() <= RESID_TOL
    assert errs.max() <= FP32_ELEM_TOL


def _whole_body_all(out, batch):
    errs, res, st = oracle_check_all(batch, out, as_f32=True)
    describe("whole-body, every instance", errs, res)
    assert not st.any()
    assert res.max() <= RESID_TOL
    assert errs.max() <= FP32_ELEM_TOL


def test_whole_body_full_batch_default_mapping():
    """n=36, m=12, N=100, batch 4096 on the default mapping, one refinement
    sweep: every instance against the oracle."""
    batch = synth.gen_batch(synth.gen_c3, 4096, np.float32)
    say("[whole-body fp32 refined] N=100 n=36 m=12 batch=4096, default mapping")
    out = run(batch, np.float32, want_resid=True, refine=1)
    assert not out["status"].any()
    say(f"  max gpu resid {out['resid'].max():.2e}")
    assert out["resid"].max() <= RESID_TOL
    _whole_body_all(out, batch)


def test_whole_body_plain_fp64_sample():
    batch = synth.gen_batch(synth.gen_c3, 64, np.float64)
    say("[whole-body plain fp64] N=100 n=36 m=12 batch=64")
    out = run(batch, np.float64, method="plain", want_resid=True)
    assert not out["status"].any()
    errs, res, _ = oracle_check_all(batch, out)
    assert errs.max() <= FP64_ELEM_TOL and res.max() <= 1e-11


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_value_function_and_policy_match_oracle(dtype):
    """P_k, p_k (the reverse scan's complete suffixes) and K_k, kff_k (the
    policy) read back from the workspace against the oracle's Riccati
    factors, element by element, on the balanced tree and on the chunked
    schedule."""
    import torch
    import oracle
    import paper_2506_07823_amd as L
    N, n, m, count = 21, 9, 4, 3
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[260, i]), count, dtype)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    tol = FP64_ELEM_TOL if dtype == np.float64 else 2e-4
    for mapping in ({}, {"engine": "wavefront", "fused": 0, "split": 2, "chunk": 4, "sweep": 6}):
        say(f"[factors {np.dtype(dtype).name}] N={N} n={n} m={m} mapping={mapping or 'default'}")
        if mapping:
            L.set_tuning(count, N, n, m, tdt, **mapping)
        try:
            dev = to_dev(batch, dtype)
            ws = L.Workspace()
            out = L.solve(*[dev[k] for k in L.FIELDS], workspace=ws, refine=0)
            fac = L.factors(count, N, n, m, tdt, ws)
            torch.cuda.synchronize()
        finally:
            if mapping:
                L.set_tuning(count, N, n, m, tdt, clear=True)
        assert not out["status"].any()
        for b in range(count):
            prob = synth.instance(batch, b)
            if dtype == np.float32:
                prob = {k: v.astype(np.float64) for k, v in prob.items()}
            ref = oracle.riccati(prob, want_factors=True)
            for f in ("P", "p", "K", "kff"):
                got = fac[f][b].cpu().numpy()
                e = max(float(np.max(np.abs(got[k] - ref[f][k]) / (np.abs(ref[f][k]) + np.abs(ref[f][k]).max())))
                        for k in range(ref[f].shape[0]))
                assert e <= tol, (mapping, b, f, e)


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
    errs, res, _ = oracle_check_all(batch, out)
    assert errs.max() <= FP64_ELEM_TOL and res.max() <= 1e-11
    for b in (3, 150):
        alone = run({k: v[b:b + 1] for k, v in b32.items()}, np.float32, refine=2, want_resid=True)
        for f in ("x", "u", "lam", "resid"):
            assert np.array_equal(alone[f][0], full[f][b]), f
