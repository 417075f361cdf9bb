"""Ragged batches through the persistent device-descriptor form
(lqr_kkt_solve_ragged_dev): problems of mixed (N, n, m) share launches, one
workgroup per problem takes them from an atomic counter.  Every result meets
the oracle (FP64 element-wise 1e-9; FP32 residual and element-wise gates),
a problem gives the same bits alone and in any mix, malformed descriptors
are flagged, the FP64 redo covers marked problems, warm starts work, and a
captured graph replays with new descriptor-table contents."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import FP32_ELEM_TOL, FP64_ELEM_TOL, RESID_TOL, elem_err, say

pytestmark = pytest.mark.gpu

SHAPES = [(25, 12, 12), (50, 36, 12), (7, 3, 2), (100, 36, 12), (13, 8, 3), (16, 4, 2), (9, 20, 9), (3, 64, 64)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401


def _problems(dtype, count=40, seed=0, shapes=SHAPES):
    rng = np.random.default_rng([970, seed])
    probs = []
    for i in range(count):
        N, n, m = shapes[int(rng.integers(0, len(shapes)))]
        probs.append(synth.as_dtype(synth.gen_rand(N, n, m, seed=[971, seed, i]), dtype))
    return probs


def _dev(p, dtype):
    import torch
    td = torch.float32 if dtype == np.float32 else torch.float64
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0", td) for k, v in p.items()}


def _oracle(p, dtype):
    import oracle
    prob = {k: np.asarray(v).astype(np.float64) for k, v in p.items()}
    return prob, oracle.riccati(prob)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_ragged_dev_meets_oracle(dtype):
    import torch
    import oracle
    import paper_2506_07823_amd as L
    probs = _problems(dtype)
    say(f"[ragged dev {np.dtype(dtype).name}] {len(probs)} problems of {len(SHAPES)} shapes")
    outs, status, resid = L.solve_ragged_dev([_dev(p, dtype) for p in probs], slots=16, want_resid=True)
    torch.cuda.synchronize()
    assert not status.any().item(), status
    worst = 0.0
    for i, p in enumerate(probs):
        prob, ref = _oracle(p, dtype)
        got = {f: outs[i][f].cpu().numpy().astype(np.float64) for f in ("x", "u", "lam")}
        e = max(elem_err(got[f], ref[f]) for f in ("x", "u", "lam"))
        res = oracle.rel_kkt_residual(prob, got["x"], got["u"], got["lam"])
        worst = max(worst, e)
        if dtype == np.float64:
            assert e <= FP64_ELEM_TOL and res <= 1e-11, (i, e, res)
        else:
            assert res <= RESID_TOL and resid[i].item() <= RESID_TOL and e <= FP32_ELEM_TOL, (i, e, res)
    say(f"  worst element-wise error {worst:.2e}")


def test_ragged_dev_alone_equals_in_mix():
    """The arithmetic of a problem does not depend on the problems beside it
    or on the workgroup that takes it."""
    import torch
    import paper_2506_07823_amd as L
    probs = _problems(np.float32, count=30, seed=1)
    dev = [_dev(p, np.float32) for p in probs]
    say("[ragged dev alone vs mix] 30 problems, 8 slots")
    outs, status, resid = L.solve_ragged_dev(dev, slots=8, want_resid=True)
    torch.cuda.synchronize()
    for i in (0, 7, 29):
        a, st, rs = L.solve_ragged_dev([dev[i]], slots=1, want_resid=True)
        torch.cuda.synchronize()
        for f in ("x", "u", "lam"):
            assert torch.equal(a[0][f], outs[i][f]), (i, f)
        assert st[0].item() == status[i].item() and rs[0].item() == resid[i].item()


def test_ragged_dev_flags_bad_descriptors_and_skips_empty():
    import torch
    import paper_2506_07823_amd as L
    shapes = [(10, 4, 2), (10, 80, 4), (10, 4, 2), (0, 4, 2)]
    descs, nin, nout = L.ragged_layout([(max(N, 1), n, m) for N, n, m in shapes])
    descs[3]["N"] = 0                          # an empty slot of a fixed-size table
    probs = [synth.as_dtype(synth.gen_rand(max(N, 1), n, m, seed=[972, i]), np.float32)
             for i, (N, n, m) in enumerate(shapes)]
    inbuf = torch.zeros(nin, dtype=torch.float32, device="cuda:0")
    for p, d in zip(probs, descs):
        for f, name in enumerate(L.FIELDS):
            t = torch.from_numpy(np.ascontiguousarray(p[name]).reshape(-1)).to("cuda:0")
            inbuf[int(d["in_off"][f]):int(d["in_off"][f]) + t.numel()].copy_(t)
    outbuf = torch.zeros(nout, dtype=torch.float32, device="cuda:0")
    status = torch.full((4,), 77, dtype=torch.int32, device="cuda:0")
    dtab = torch.from_numpy(descs.view(np.uint8).copy()).to("cuda:0")
    say("[ragged dev bad descriptors]")
    L.solve_ragged_packed(dtab, inbuf, outbuf, status, count=4, slots=4, maxN=10, maxd=64)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[0] == 0 and st[2] == 0, st
    assert st[1] == L.ST_BAD_DESC, st          # order 80: no wavefront class
    assert st[3] == L.ST_BAD_DESC, st          # N = 0 is not a problem


def test_ragged_dev_fallback():
    import torch
    import oracle
    import paper_2506_07823_amd as L
    probs = _problems(np.float32, count=6, seed=2, shapes=[(12, 8, 4)])
    probs[3]["R"][5] = np.diag([1e-7, 1.0, 1.0, 1.0]).astype(np.float32)
    say("[ragged dev fallback] cond(R) = 1e7 in problem 3")
    outs, status, resid = L.solve_ragged_dev([_dev(p, np.float32) for p in probs], slots=4, want_resid=True)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[3] == 8 and not np.delete(st, 3).any(), st
    prob, ref = _oracle(probs[3], np.float32)
    got = {f: outs[3][f].cpu().numpy().astype(np.float64) for f in ("x", "u", "lam")}
    res = oracle.rel_kkt_residual(prob, got["x"], got["u"], got["lam"])
    say(f"  redone problem: resid gpu {resid[3].item():.2e} oracle {res:.2e}")
    assert res <= RESID_TOL and resid[3].item() <= RESID_TOL


def test_ragged_dev_warm_start_and_graph_replay_with_new_table():
    """Capture one ragged call into a graph, then replay it after writing a
    different problem mix (same count) into the same buffers: the replay
    solves the new problems.  A warm-started call (from the cold solution of
    slightly changed initial states) meets the residual gate."""
    import torch
    import paper_2506_07823_amd as L
    count = 12
    mixes = [_problems(np.float32, count=count, seed=s, shapes=SHAPES[:6]) for s in (3, 4)]
    layouts = [L.ragged_layout([p["B"].shape for p in mix]) for mix in mixes]
    nin = max(l[1] for l in layouts)
    nout = max(l[2] for l in layouts)
    inbuf = torch.zeros(nin, dtype=torch.float32, device="cuda:0")
    outbuf = torch.zeros(nout, dtype=torch.float32, device="cuda:0")
    dtab = torch.zeros(count * L.DESC_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
    status = torch.zeros(count, dtype=torch.int32, device="cuda:0")
    resid = torch.zeros(count, dtype=torch.float64, device="cuda:0")
    ws = L.Workspace()
    kw = dict(count=count, slots=8, maxN=100, maxd=36, resid=resid, workspace=ws)

    def load(mix, lay):
        descs = lay[0]
        inbuf.zero_()
        for p, d in zip(mix, descs):
            for f, name in enumerate(L.FIELDS):
                t = torch.from_numpy(np.ascontiguousarray(p[name]).reshape(-1)).to("cuda:0")
                inbuf[int(d["in_off"][f]):int(d["in_off"][f]) + t.numel()].copy_(t)
        dtab.copy_(torch.from_numpy(descs.view(np.uint8).copy()))

    load(mixes[0], layouts[0])
    L.solve_ragged_packed(dtab, inbuf, outbuf, status, **kw)     # sizes the workspace
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        L.solve_ragged_packed(dtab, inbuf, outbuf, status, **kw)
    torch.cuda.synchronize()
    for mix, lay in zip(mixes, layouts):
        load(mix, lay)
        torch.cuda.synchronize()
        say(f"[ragged dev graph replay] shapes {[tuple(p['B'].shape) for p in mix][:4]} ...")
        g.replay()
        torch.cuda.synchronize()
        ref_out, ref_st, ref_rs = L.solve_ragged_dev([_dev(p, np.float32) for p in mix], slots=8, want_resid=True)
        torch.cuda.synchronize()
        assert not status.any().item() and resid.max().item() <= RESID_TOL
        for i, d in enumerate(lay[0]):
            for f, name in enumerate(("x", "u", "lam")):
                off = int(d["out_off"][f])
                seg = outbuf[off:off + ref_out[i][name].numel()]
                assert torch.equal(seg, ref_out[i][name].reshape(-1)), (i, name)
    # warm start: the last mix with perturbed x0, from the solution above
    mix, lay = mixes[1], layouts[1]
    rng = np.random.default_rng(5)
    for p in mix:
        p["x0"] = (p["x0"] + rng.normal(0, 1e-2, p["x0"].shape)).astype(np.float32)
    load(mix, lay)
    warm = outbuf.clone()
    L.solve_ragged_packed(dtab, inbuf, outbuf, status, warm=(warm, warm, warm), **kw)
    torch.cuda.synchronize()
    say(f"  warm-started: max resid {resid.max().item():.2e}")
    assert not status.any().item() and resid.max().item() <= RESID_TOL
