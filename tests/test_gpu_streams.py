"""Batch split over streams (mapping field `streams`): the parts' launch
sequences run on streams forked from the caller's and joined back, and
every instance gets the same bits as in the one-stream solve of the same
mapping (an instance's arithmetic does not depend on the part it is in).
Checked against the oracle element-wise, for part sizes that do not divide
the batch, under graph replay with new inputs between replays, for the
re-solve, the factor read-back, an in-place warm start, the no-allocation
entry point and a tuning-cache line carrying the field."""
import ctypes

import numpy as np
import pytest

import synth
from tests.gpuhelp import FP32_ELEM_TOL, FP64_ELEM_TOL, RESID_TOL, oracle_check_all, say, to_dev

pytestmark = pytest.mark.gpu

SEQ = {"engine": "wavefront", "fused": 0, "split": 2, "chunk": 1, "sweep": 1, "fwd_seq": True}
MAPPINGS = [{"engine": "wavefront", "fused": 0}, SEQ, {"engine": "wavefront", "fused": 2},
            {"engine": "matrix-core", "fused": 0}]
OUTS = ("x", "u", "lam", "status", "resid")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401


def _shape(batch):
    count, N, n, _ = batch["A"].shape
    return count, N, n, batch["B"].shape[-1]


def _tdt(dtype):
    import torch
    return torch.float32 if dtype == np.float32 else torch.float64


def _solve(batch, dtype, mapping, streams, **kw):
    import torch
    import paper_2506_07823_amd as L
    count, N, n, m = _shape(batch)
    L.set_tuning(count, N, n, m, _tdt(dtype), streams=streams, **mapping)
    try:
        dev = to_dev(batch, dtype)
        out = L.solve(*[dev[k] for k in L.FIELDS], want_resid=True, **kw)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        L.set_tuning(count, N, n, m, _tdt(dtype), clear=True)


def _same(a, b):
    for f in OUTS:
        assert np.array_equal(a[f], b[f]), f


@pytest.mark.parametrize("mapping", MAPPINGS)
@pytest.mark.parametrize("count,streams", [(7, 4), (8, 2), (5, 3)])
def test_split_equals_one_stream_fp64(mapping, count, streams):
    N, n, m = 12, 40, 12
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[990, count, i]), count, np.float64)
    say(f"[streams fp64] batch={count} streams={streams} {mapping}")
    one = _solve(batch, np.float64, mapping, 0)
    split = _solve(batch, np.float64, mapping, streams)
    _same(one, split)
    assert not split["status"].any()
    errs, res, _ = oracle_check_all(batch, split)
    assert errs.max() <= FP64_ELEM_TOL and res.max() <= 1e-11, errs


@pytest.mark.parametrize("streams", [2, 4])
def test_split_whole_body_fp32(streams):
    batch = synth.gen_batch(synth.gen_c3, 510, np.float32)
    say(f"[streams fp32 whole-body] batch=510 streams={streams}")
    one = _solve(batch, np.float32, SEQ, 0, refine=1)
    split = _solve(batch, np.float32, SEQ, streams, refine=1)
    _same(one, split)
    assert not split["status"].any()
    errs, res, _ = oracle_check_all(batch, split, as_f32=True)
    say(f"  element-wise err max {errs.max():.2e}, oracle resid max {res.max():.2e}")
    assert res.max() <= RESID_TOL and split["resid"].max() <= RESID_TOL and errs.max() <= FP32_ELEM_TOL


def test_split_under_graph_replay():
    """A captured split solve, replayed with new inputs copied into its
    buffers and eager work between replays, equals the eager solve of each
    input set."""
    import torch
    import paper_2506_07823_amd as L
    sets = [synth.gen_batch(lambda i, s=s: synth.gen_c3(1000 * s + i), 96, np.float32) for s in range(3)]
    count, N, n, m = _shape(sets[0])
    L.set_tuning(count, N, n, m, torch.float32, streams=3, **SEQ)
    try:
        eager = []
        for b in sets:
            dev = to_dev(b, np.float32)
            o = L.solve(*[dev[k] for k in L.FIELDS], want_resid=True, refine=1)
            torch.cuda.synchronize()
            eager.append({k: v.cpu().numpy() for k, v in o.items()})
        dev = to_dev(sets[0], np.float32)
        ws = L.Workspace()
        out = L.solve(*[dev[k] for k in L.FIELDS], want_resid=True, refine=1, workspace=ws)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            L.solve(*[dev[k] for k in L.FIELDS], want_resid=True, refine=1, workspace=ws, out=out, stream=s)
        torch.cuda.synchronize()
        for rep in range(6):
            j = rep % 3
            host = to_dev(sets[j], np.float32)
            for k in L.FIELDS:
                dev[k].copy_(host[k])
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = {k: v.cpu().numpy() for k, v in out.items()}
            say(f"  replay {rep}: input set {j}")
            _same(got, eager[j])
            # eager work between replays
            L.solve(*[host[k] for k in L.FIELDS], refine=1)
            torch.cuda.synchronize()
    finally:
        L.set_tuning(count, N, n, m, torch.float32, clear=True)


def test_split_resolve_and_factors():
    """The re-solve and the factor read-back find each part's records in its
    workspace slice: both equal the one-stream results."""
    import torch
    import paper_2506_07823_amd as L
    N, n, m = 20, 12, 4
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[991, i]), 7, np.float64)
    rng = np.random.default_rng(992)
    nb = {k: v.copy() for k, v in batch.items()}
    for f in ("x0", "q", "r"):
        nb[f] = nb[f] + rng.normal(0, 0.1, nb[f].shape)
    res = []
    for streams in (0, 3):
        L.set_tuning(7, N, n, m, torch.float64, streams=streams, **SEQ)
        try:
            dev = to_dev(batch, np.float64)
            ws = L.Workspace()
            out = L.solve(*[dev[k] for k in L.FIELDS], workspace=ws, want_resid=True)
            fac = L.factors(7, N, n, m, torch.float64, ws)
            dev2 = to_dev(nb, np.float64)
            L.resolve(*[dev2[k] for k in L.FIELDS], out=out, workspace=ws, want_resid=True)
            torch.cuda.synchronize()
            res.append(({k: v.cpu().numpy() for k, v in out.items()}, {k: v.cpu().numpy() for k, v in fac.items()}))
        finally:
            L.set_tuning(7, N, n, m, torch.float64, clear=True)
    _same(res[0][0], res[1][0])
    for f in ("P", "p", "K", "kff"):
        assert np.array_equal(res[0][1][f], res[1][1][f]), f
    errs, r, _ = oracle_check_all(nb, res[1][0])
    assert errs.max() <= FP64_ELEM_TOL and r.max() <= 1e-11


def test_split_in_place_warm_start():
    import torch
    import paper_2506_07823_amd as L
    batch = synth.gen_batch(synth.gen_c3, 64, np.float32)
    got = []
    for streams in (0, 4):
        L.set_tuning(64, 100, 36, 12, torch.float32, streams=streams, **SEQ)
        try:
            dev = to_dev(batch, np.float32)
            out = L.solve(*[dev[k] for k in L.FIELDS], refine=1, want_resid=True)
            L.solve(*[dev[k] for k in L.FIELDS], refine=1, want_resid=True, warm=(out["x"], out["u"], out["lam"]),
                    out=out)
            torch.cuda.synchronize()
            got.append({k: v.cpu().numpy() for k, v in out.items()})
        finally:
            L.set_tuning(64, 100, 36, 12, torch.float32, clear=True)
    _same(got[0], got[1])
    assert got[1]["resid"].max() <= RESID_TOL and not got[1]["status"].any()


def test_split_no_alloc_entry_point():
    import torch
    import paper_2506_07823_amd as L
    N, n, m = 50, 12, 12
    batch = synth.gen_batch(lambda i: synth.gen_c2(N, i), 6, np.float32)
    ref = _solve(batch, np.float32, SEQ, 0)
    L.set_tuning(6, N, n, m, torch.float32, streams=4, **SEQ)
    try:
        dev = to_dev(batch, np.float32)
        out = {"x": torch.zeros((6, N + 1, n), device="cuda:0"), "u": torch.zeros((6, N, m), device="cuda:0"),
               "lam": torch.zeros((6, N + 1, n), device="cuda:0"),
               "status": torch.full((6,), 99, dtype=torch.int32, device="cuda:0"),
               "resid": torch.zeros((6,), dtype=torch.float64, device="cuda:0")}
        o = L.default_opts(torch.float32)
        o.resid_out = out["resid"].data_ptr()
        s = torch.cuda.current_stream().cuda_stream
        rc = L.lqr_kkt_solve_noalloc(L.handle(0), s, 6, N, n, m, *[dev[k].data_ptr() for k in L.FIELDS],
                                     out["x"].data_ptr(), out["u"].data_ptr(), out["lam"].data_ptr(),
                                     out["status"].data_ptr(), ctypes.byref(o))
        assert rc == 0, L.lqr_last_error()
        torch.cuda.synchronize()
        _same(ref, {k: v.cpu().numpy() for k, v in out.items()})
    finally:
        L.set_tuning(6, N, n, m, torch.float32, clear=True)


def test_tuning_cache_line_with_streams(tmp_path):
    """A cache line with the streams field is loaded for its bucket and the
    solve of that shape runs split (same bits as the pinned one-stream
    solve); a line without it still loads."""
    import torch
    import paper_2506_07823_amd as L
    N, n, m = 20, 12, 4
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[993, i]), 6, np.float32)
    ref = _solve(batch, np.float32, SEQ, 0)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = tmp_path / "tune.txt"
    # dtype 0 = FP32; buckets N 32, batch 8; wavefront, fused 0, chunked 1/1, fwd_seq, 4 streams
    path.write_text(f"lqr-tune-1 {arch} 0 {n} {m} 32 8 1 0 0 2 1 1 1 4\n"
                    f"lqr-tune-1 {arch} 0 {n} {m} 32 16 1 0 0 2 1 1 1\n")
    assert L.load_tuning(str(path)) == 2
    dev = to_dev(batch, np.float32)
    out = L.solve(*[dev[k] for k in L.FIELDS], want_resid=True)
    torch.cuda.synchronize()
    _same(ref, {k: v.cpu().numpy() for k, v in out.items()})
    L.save_tuning(str(path))
    lines = path.read_text().splitlines()
    say(f"[tuning cache] {lines}")
    assert f"lqr-tune-1 {arch} 0 {n} {m} 32 8 1 0 0 2 1 1 1 4" in lines
    for Bb in (8, 16):
        L.set_tuning(Bb, 32, n, m, torch.float32, clear=True)
