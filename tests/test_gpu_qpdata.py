"""QP-data builder on the GPU (lqr_qp_build, Sec. II-F) against the oracle
of oracle/qpdata.py, element by element, and end to end: the blocks built
on the GPU, solved on the GPU, match the oracle's blocks solved by the
oracle."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import FP64_ELEM_TOL, elem_err_batch, oracle_check_all, say

pytestmark = pytest.mark.gpu

BLOCKS = ("Q", "M", "R", "q", "r")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401


def _build(d, dtype):
    import torch
    import paper_2506_07823_amd as L
    td = torch.float32 if dtype == np.float32 else torch.float64
    dev = {k: torch.from_numpy(np.ascontiguousarray(d[k], dtype=dtype)).to("cuda:0", td)
           for k in synth.QP_FIELDS + ("mu", "delta")}
    nc = d["Gx"].shape[-2]
    args = [dev[k] for k in ("Ex", "Eu", "e", "W")]
    if nc:
        args += [dev[k] for k in ("Gx", "Gu", "g", "mu", "delta")]
    out = L.qp_build(*args)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("N,n,m,nc", [(10, 4, 2, 3), (25, 12, 12, 8), (20, 36, 12, 24), (5, 36, 12, 0)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_qp_build_matches_oracle(N, n, m, nc, dtype):
    from oracle import qpdata
    d = synth.gen_qp_batch(4, N, n, m, nc, [990, N, n, m, nc])
    if dtype == np.float32:
        d = {k: v.astype(np.float32).astype(np.float64) for k, v in d.items()}
    if nc == 0:
        d["Gx"] = np.zeros((4, N + 1, 0, n))
        d["Gu"] = np.zeros((4, N, 0, m))
        d["g"] = np.zeros((4, N + 1, 0))
        d["mu"] = np.zeros(0)
        d["delta"] = np.zeros(0)
    say(f"[qp build {np.dtype(dtype).name}] N={N} n={n} m={m} p={n + m} nc={nc}")
    got = _build(d, dtype)
    ref = qpdata.build(d)
    tol = FP64_ELEM_TOL if dtype == np.float64 else 2e-5
    for k in BLOCKS:
        err = elem_err_batch(got[k], ref[k]).max()
        say(f"  {k}: element-wise err {err:.2e}")
        assert err <= tol, (k, err)


def test_built_qp_solves_like_the_oracle():
    """GPU-built blocks + the dynamics, solved by the GPU scan in FP64, match
    the oracle's Riccati solve of the oracle-built blocks."""
    import torch
    import paper_2506_07823_amd as L
    from oracle import qpdata
    N, n, m, nc = 30, 12, 12, 8
    d = synth.gen_qp_batch(3, N, n, m, nc, [991])
    say(f"[qp build -> solve] N={N} n={n} m={m} nc={nc}")
    got = _build(d, np.float64)
    ref = qpdata.build(d)
    prob = {"A": d["A"], "B": d["B"], "c": d["c"], "x0": d["x0"], **ref}
    dev = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to("cuda:0") for k in ("A", "B", "c", "x0")}
    dev.update({k: torch.from_numpy(np.ascontiguousarray(got[k])).to("cuda:0") for k in BLOCKS})
    out = L.solve(*[dev[k] for k in L.FIELDS])
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    assert not out["status"].any()
    errs, res, _ = oracle_check_all(prob, out)
    assert errs.max() <= FP64_ELEM_TOL and res.max() <= 1e-11, errs
