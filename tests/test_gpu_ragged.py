"""Ragged batches through the C ABI: one call with problems of mixed
(N, n, m), in scrambled order, returns for every problem exactly what solving
it alone returns (same per-instance arithmetic), with status and residual in
descriptor order; FP64 results meet the oracle bar."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import oracle_check, rel, run, say

pytestmark = pytest.mark.gpu

SHAPES = [(25, 12, 12), (50, 36, 12), (7, 3, 2), (6, 70, 20), (13, 8, 3)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401


def _problems(dtype, count=23, seed=0):
    rng = np.random.default_rng([900, seed])
    probs = []
    for i in range(count):
        N, n, m = SHAPES[int(rng.integers(0, len(SHAPES)))]
        probs.append(synth.as_dtype(synth.gen_rand(N, n, m, seed=[901, seed, i]), dtype))
    return probs


def _dev(p, dtype):
    import torch
    td = torch.float32 if dtype == np.float32 else torch.float64
    return {k: torch.from_numpy(v).to("cuda:0", td) for k, v in p.items()}


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_ragged_equals_alone(dtype):
    import torch
    import paper_2506_07823_amd as L
    probs = _problems(dtype)
    say(f"[ragged {np.dtype(dtype).name}] {len(probs)} problems of {len(SHAPES)} shapes")
    outs, status, resid = L.solve_ragged([_dev(p, dtype) for p in probs], want_resid=True)
    torch.cuda.synchronize()
    assert not status.any().item(), status
    for i, p in enumerate(probs):
        alone = run({k: v[None] for k, v in p.items()}, dtype, want_resid=True)
        for f in ("x", "u", "lam"):
            assert np.array_equal(outs[i][f].cpu().numpy(), alone[f][0]), (i, f)
        assert resid[i].item() == alone["resid"][0]
    if dtype == np.float64:
        for i in (0, 5, 22):
            b = {k: v[None] for k, v in probs[i].items()}
            o = {f: outs[i][f].cpu().numpy()[None] for f in ("x", "u", "lam")}
            errs, res = oracle_check(b, o, 0)
            assert max(errs) <= 1e-9 and res <= 1e-11
    else:
        assert resid.max().item() <= 1e-5


def test_ragged_status_in_descriptor_order():
    import torch
    import paper_2506_07823_amd as L
    probs = _problems(np.float64, count=9, seed=1)
    probs[4]["R"][0] = -100.0 * np.eye(probs[4]["R"].shape[-1])   # indefinite R in problem 4 only
    say("[ragged status] indefinite R in problem 4")
    outs, status, _ = L.solve_ragged([_dev(p, np.float64) for p in probs], refine=0)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[4] & 2 and (np.delete(st, 4) == 0).all(), st


def test_ragged_rejects_bad_descriptor_before_launch():
    import paper_2506_07823_amd as L
    probs = [_dev(p, np.float32) for p in _problems(np.float32, count=3, seed=2)]
    probs[1]["B"] = probs[1]["B"][..., :-1].contiguous()   # inconsistent shapes
    with pytest.raises(ValueError):
        L.solve_ragged(probs)
