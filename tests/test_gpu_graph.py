"""The solve captured into a HIP graph replays to the eager result.

The whole launch sequence (fill kernel for status/queue counters, scan,
policy, forward scan, refinement, residual) is captured once and replayed
several times, with eager work and synchronizations between the replays;
every replay is compared bitwise with the eager solve."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("cfg", ["srbd50_fp32", "wholebody_fp32", "tiny_fp64_plain", "matrixcore_fp32",
                                 "matrixcore_fp64_plain"])
def test_graph_replay_matches_eager(cfg):
    import torch
    import paper_2506_07823_amd as L
    if cfg == "srbd50_fp32":
        batch, dt, kw = synth.gen_batch(lambda i: synth.gen_c2(50, i), 4, np.float32), np.float32, {}
    elif cfg == "wholebody_fp32":
        batch, dt, kw = synth.gen_batch(synth.gen_c3, 32, np.float32), np.float32, {}
    elif cfg == "matrixcore_fp32":
        batch = synth.gen_batch(lambda i: synth.gen_rand(6, 80, 40, seed=[850, i]), 3, np.float32)
        dt, kw = np.float32, {}
    elif cfg == "matrixcore_fp64_plain":
        batch = synth.gen_batch(lambda i: synth.gen_rand(5, 72, 24, seed=[851, i]), 2, np.float64)
        dt, kw = np.float64, {"method": "plain"}
    else:
        batch, dt, kw = synth.gen_batch(synth.gen_c1, 3, np.float64), np.float64, {"method": "plain"}
    say(f"[graph replay] {cfg}")
    dev = to_dev(batch, dt)
    args = [dev[k] for k in L.FIELDS]
    eager = L.solve(*args, want_resid=True, **kw)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in eager.items()}
    ws = L.Workspace()
    out = L.solve(*args, want_resid=True, workspace=ws, **kw)      # sizes the workspace
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):     # captures on torch's side stream (the current stream inside)
        L.solve(*args, want_resid=True, workspace=ws, out=out, **kw)
    torch.cuda.synchronize()
    for rep in range(4):
        for v in out.values():          # eager work between replays
            v.fill_(-1)
        ws.buf.fill_(0x7f)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ("x", "u", "lam", "status", "resid"):
            assert torch.equal(out[k], ref[k]), (rep, k)
