"""Re-solve with cached factors (lqr_kkt_resolve): after a scan solve, new
(x0, c, q, r) with the same matrices are solved from the value function,
policy and closed-loop matrices left in the workspace.  Checked against the
oracle on the new problem (FP64 element-wise 1e-9, FP32 residual and
element-wise gates) on every mapping family, bit for bit against itself on
repeat, and with an instance the FP64 fallback solved."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import FP32_ELEM_TOL, FP64_ELEM_TOL, RESID_TOL, oracle_check_all, say, to_dev

pytestmark = pytest.mark.gpu

MAPPINGS = [None, {"engine": "wavefront", "fused": 0, "split": 2, "chunk": 1, "sweep": 1, "fwd_seq": True},
            {"engine": "wavefront", "fused": 1}, {"engine": "wavefront", "fused": 2},
            {"engine": "matrix-core", "fused": 0}]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401


def _new_rhs(batch, seed):
    rng = np.random.default_rng(seed)
    nb = {k: v.copy() for k, v in batch.items()}
    for f, s in (("x0", 0.1), ("c", 1e-3), ("q", 1.0), ("r", 1.0)):
        nb[f] = (nb[f] + rng.normal(0, s, nb[f].shape)).astype(nb[f].dtype)
    return nb


def _solve_then_resolve(batch, nb, dtype, mapping, **kw):
    import torch
    import paper_2506_07823_amd as L
    count, N, n, _ = batch["A"].shape
    m = batch["B"].shape[-1]
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    if mapping:
        L.set_tuning(count, N, n, m, tdt, **mapping)
    try:
        dev = to_dev(batch, dtype)
        ws = L.Workspace()
        out = L.solve(*[dev[k] for k in L.FIELDS], workspace=ws, want_resid=True, **kw)
        dev2 = to_dev(nb, dtype)
        L.resolve(*[dev2[k] for k in L.FIELDS], out=out, workspace=ws, want_resid=True, **kw)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        if mapping:
            L.set_tuning(count, N, n, m, tdt, clear=True)


@pytest.mark.parametrize("mapping", MAPPINGS)
@pytest.mark.parametrize("N,n,m", [(16, 4, 2), (30, 12, 12), (11, 36, 12)])
def test_resolve_fp64_meets_oracle(mapping, N, n, m):
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[980, N, n, m, i]), 3, np.float64)
    nb = _new_rhs(batch, [981, N])
    say(f"[resolve fp64] N={N} n={n} m={m} {mapping or 'default'}")
    out = _solve_then_resolve(batch, nb, np.float64, mapping)
    assert not out["status"].any(), out["status"]
    errs, res, _ = oracle_check_all(nb, out)
    assert errs.max() <= FP64_ELEM_TOL and res.max() <= 1e-11, errs


@pytest.mark.parametrize("mapping", MAPPINGS[:2])
def test_resolve_fp32_whole_body(mapping):
    batch = synth.gen_batch(synth.gen_c3, 256, np.float32)
    nb = _new_rhs(batch, [982])
    say(f"[resolve fp32 whole-body] batch=256 {mapping or 'default'}")
    out = _solve_then_resolve(batch, nb, np.float32, mapping, refine=1)
    assert not out["status"].any()
    errs, res, _ = oracle_check_all(nb, out, as_f32=True)
    say(f"  element-wise err max {errs.max():.2e}, oracle resid max {res.max():.2e}, gpu {out['resid'].max():.2e}")
    assert res.max() <= RESID_TOL and out["resid"].max() <= RESID_TOL and errs.max() <= FP32_ELEM_TOL


def test_resolve_redoes_fallback_instance():
    N, n, m = 12, 8, 4
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[983, i]), 3, np.float32)
    batch["R"][1, 5] = np.diag([1e-7, 1.0, 1.0, 1.0])
    nb = _new_rhs(batch, [984])
    say("[resolve fallback]")
    out = _solve_then_resolve(batch, nb, np.float32, None)
    assert out["status"][1] == 8 and out["status"][0] == 0 and out["status"][2] == 0, out["status"]
    errs, res, _ = oracle_check_all(nb, out, as_f32=True)
    assert res.max() <= RESID_TOL, res


def test_resolve_rejects_other_methods():
    import torch
    import paper_2506_07823_amd as L
    b = synth.gen_batch(lambda i: synth.gen_rand(5, 4, 2, seed=[985, i]), 2, np.float32)
    dev = to_dev(b, np.float32)
    ws = L.Workspace()
    out = L.solve(*[dev[k] for k in L.FIELDS], workspace=ws)
    torch.cuda.synchronize()
    with pytest.raises(L.LqrError):
        L.resolve(*[dev[k] for k in L.FIELDS], out=out, workspace=ws, refine=9)
