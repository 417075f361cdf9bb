"""Chunked schedule of the reverse scan (mapping split = 2: a sequential
sweep over the last `sweep` elements, chunks of `chunk` elements over the
others) and the sequential vector passes (fwd_seq = 1: forward scan,
recovery and refinement as sweeps over the stages), against the oracle:
FP64 element-wise to 1e-9, FP32 to the residual and element-wise gates,
every instance of the full whole-body batch, graph replay, the FP64 redo of
a marked instance, and the rejected mappings."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import (FP32_ELEM_TOL, FP64_ELEM_TOL, RESID_TOL, describe, oracle_check, oracle_check_all, say,
                           to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401


def _pinned(batch, dtype, mapping, **kw):
    import torch
    import paper_2506_07823_amd as L
    count, N, n, _ = batch["A"].shape
    m = batch["B"].shape[-1]
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    L.set_tuning(count, N, n, m, tdt, **mapping)
    try:
        dev = to_dev(batch, dtype)
        out = L.solve(*[dev[k] for k in L.FIELDS], **kw)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        L.set_tuning(count, N, n, m, tdt, clear=True)


def _chunked(chunk, sweep, fwd_seq=False):
    return {"engine": "wavefront", "fused": 0, "split": 2, "chunk": chunk, "sweep": sweep, "fwd_seq": fwd_seq}


SHAPES = [(1, 4, 2), (7, 3, 2), (13, 8, 3), (25, 12, 12), (40, 36, 12)]
SCHEDS = [(1, 1), (4, 1), (3, 5), (8, 10 ** 6), (16, 2)]


@pytest.mark.parametrize("N,n,m", SHAPES)
@pytest.mark.parametrize("chunk,sweep", SCHEDS)
@pytest.mark.parametrize("fwd_seq", [False, True])
def test_chunked_fp64_meets_oracle(N, n, m, chunk, sweep, fwd_seq):
    sweep = min(sweep, N + 1)
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[960, N, n, m, i]), 3, np.float64)
    say(f"[chunked fp64] N={N} n={n} m={m} chunk={chunk} sweep={sweep} fwd_seq={fwd_seq}")
    out = _pinned(batch, np.float64, _chunked(chunk, sweep, fwd_seq))
    assert not out["status"].any(), out["status"]
    errs, res, _ = oracle_check_all(batch, out)
    assert errs.max() <= FP64_ELEM_TOL, errs
    assert res.max() <= 1e-11


# Shapes whose chunked sweeps combine each leaf through its rank-m factor
# V = B R^{-1/2} (orders 17..64 with m <= 16): factors of one and two row
# blocks, tile orders 3, 4, 5, 6 and 8, m = 1 and m = 16 at the class edges,
# a one-stage horizon (the sweep's single step starts from Q_N).
# Schedules: chunk 1 (every chunk-start suffix in the leaf form), chunks of
# 4 behind a 3-leaf sweep (the chunk interiors in the leaf form), chunk 1
# behind a 5-leaf sweep (the leaf form takes over a suffix the general form
# stored), chunks of 5 with a short last chunk.
LEAF_SHAPES = [(9, 17, 16), (20, 24, 1), (12, 40, 8), (7, 64, 16), (30, 50, 5), (1, 32, 16), (3, 17, 8)]
LEAF_SCHEDS = [(1, 1), (4, 3), (1, 5), (5, 1)]


@pytest.mark.parametrize("N,n,m", LEAF_SHAPES)
@pytest.mark.parametrize("chunk,sweep", LEAF_SCHEDS)
def test_chunked_leaf_form_fp64(N, n, m, chunk, sweep):
    sweep = min(sweep, N + 1)
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[966, N, n, m, i]), 3, np.float64)
    say(f"[chunked leaf form fp64] N={N} n={n} m={m} chunk={chunk} sweep={sweep}")
    out = _pinned(batch, np.float64, _chunked(chunk, sweep, True))
    assert not out["status"].any(), out["status"]
    errs, res, _ = oracle_check_all(batch, out)
    assert errs.max() <= FP64_ELEM_TOL, errs
    assert res.max() <= 1e-11


@pytest.mark.parametrize("N,n,m", [(60, 24, 8), (50, 48, 16), (40, 64, 3), (60, 20, 12)])
@pytest.mark.parametrize("chunk,sweep", [(1, 1), (4, 3)])
def test_chunked_leaf_form_fp32_refined(N, n, m, chunk, sweep):
    batch = synth.gen_batch(lambda i: synth.gen_c1_like(N, n, m, [967, N, n, m, i], dt=0.01), 5, np.float32)
    say(f"[chunked leaf form fp32] N={N} n={n} m={m} chunk={chunk} sweep={sweep}")
    out = _pinned(batch, np.float32, _chunked(chunk, sweep, True), want_resid=True, refine=1)
    assert not out["status"].any(), out["status"]
    errs, res, _ = oracle_check_all(batch, out, as_f32=True)
    describe(f"n={n} m={m}", errs, res)
    assert out["resid"].max() <= RESID_TOL and res.max() <= RESID_TOL
    assert errs.max() <= FP32_ELEM_TOL


@pytest.mark.parametrize("mapping", [{"engine": "wavefront", "fused": 0, "fwd_seq": True},
                                     {"engine": "wavefront", "fused": 0, "split": 1, "fwd_seq": True},
                                     {"engine": "matrix-core", "fused": 0, "fwd_seq": True}])
@pytest.mark.parametrize("N,n,m", [(16, 4, 2), (33, 12, 12), (9, 20, 9)])
def test_sequential_vector_passes_fp64(mapping, N, n, m):
    batch = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[961, N, n, m, i]), 3, np.float64)
    say(f"[fwd_seq fp64] N={N} n={n} m={m} {mapping}")
    out = _pinned(batch, np.float64, mapping)
    assert not out["status"].any(), out["status"]
    errs, res, _ = oracle_check_all(batch, out)
    assert errs.max() <= FP64_ELEM_TOL and res.max() <= 1e-11


def test_sequential_vector_passes_large_blocks_fp64():
    N, n, m = 6, 70, 12
    batch = synth.gen_batch(lambda i: synth.gen_c1_like(N, n, m, [962, i]), 2, np.float64)
    say(f"[fwd_seq fp64 large blocks] N={N} n={n} m={m}")
    out = _pinned(batch, np.float64, {"engine": "matrix-core", "fused": 0, "fwd_seq": True})
    assert not out["status"].any(), out["status"]
    errs, res, _ = oracle_check_all(batch, out)
    assert errs.max() <= FP64_ELEM_TOL and res.max() <= 1e-11


@pytest.mark.parametrize("chunk,sweep,fwd_seq", [(1, 1, True), (8, 1, True), (4, 30, False), (16, 1, False)])
@pytest.mark.parametrize("N", [50, 100])
def test_chunked_fp32_refined(chunk, sweep, fwd_seq, N):
    batch = synth.gen_batch(lambda i: synth.gen_c2(N, i), 3, np.float32)
    say(f"[chunked fp32] srbd N={N} chunk={chunk} sweep={sweep} fwd_seq={fwd_seq}")
    out = _pinned(batch, np.float32, _chunked(chunk, sweep, fwd_seq), want_resid=True, refine=1)
    assert not out["status"].any(), out["status"]
    errs, res, _ = oracle_check_all(batch, out, as_f32=True)
    describe("srbd", errs, res)
    assert out["resid"].max() <= RESID_TOL and res.max() <= RESID_TOL
    assert errs.max() <= FP32_ELEM_TOL


@pytest.mark.parametrize("chunk,sweep", [(1, 1), (8, 1)])
def test_chunked_whole_body_full_batch(chunk, sweep):
    """The whole-body batch (4096 instances, N=100) on the sequential
    schedules the benchmark's autotuner weighs, one refinement sweep: every
    instance against the oracle."""
    batch = synth.gen_batch(synth.gen_c3, 4096, np.float32)
    say(f"[chunked whole-body] batch=4096 chunk={chunk} sweep={sweep} fwd_seq=1")
    out = _pinned(batch, np.float32, _chunked(chunk, sweep, True), want_resid=True, refine=1)
    assert not out["status"].any()
    assert out["resid"].max() <= RESID_TOL
    errs, res, st = oracle_check_all(batch, out, as_f32=True)
    describe("whole-body, every instance", errs, res)
    assert not st.any()
    assert res.max() <= RESID_TOL and errs.max() <= FP32_ELEM_TOL


def test_chunked_fallback_redoes_the_instance():
    """A terminal weight with condition 3.3e6 marks the instance in the
    sequential sweep; it is solved again whole in FP64 (bit 8 only)."""
    N, n, m = 25, 12, 12
    b = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[963, i]), 3, np.float32)
    b["Q"][1, N] = np.diag([3e-3] + [1.0] * (n - 2) + [1e4])
    say("[chunked fallback]")
    out = _pinned(b, np.float32, _chunked(4, 3, True), want_resid=True)
    assert out["status"][1] == 8, out["status"]
    assert out["status"][0] == 0 and out["status"][2] == 0, out["status"]
    errs, res = oracle_check(b, out, 1, as_f32=True)
    say(f"  marked instance: elem err {errs}, resid gpu {out['resid'][1]:.2e} oracle {res:.2e}")
    assert out["resid"][1] <= 1e-5 and res <= 1e-5


def test_chunked_in_a_graph_replays_identically():
    """Replays of a captured chunked + sequential-pass solve give the eager
    bits with the outputs and the whole workspace overwritten between
    replays (nothing reads a record the solve did not write)."""
    import torch
    import paper_2506_07823_amd as L
    N, n, m, count = 30, 12, 12, 8
    b = synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[964, i]), count, np.float32)
    dev = to_dev(b, np.float32)
    args = [dev[k] for k in L.FIELDS]
    L.set_tuning(count, N, n, m, torch.float32, **_chunked(4, 5, True))
    try:
        eager = L.solve(*args, want_resid=True)
        torch.cuda.synchronize()
        ref = {k: v.clone() for k, v in eager.items()}
        ws = L.Workspace()
        out = L.solve(*args, want_resid=True, workspace=ws)
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


def test_chunked_leaf_form_in_a_graph_replays_identically():
    """Chunk length 1 at a leaf-form shape (every leaf combined through its
    rank-m factor, the elements' C parts left unwritten): replays with the
    whole workspace overwritten between them give the eager bits, so no
    kernel reads a record part the solve did not write."""
    import torch
    import paper_2506_07823_amd as L
    N, n, m, count = 40, 24, 8, 6
    b = synth.gen_batch(lambda i: synth.gen_c1_like(N, n, m, [968, i], dt=0.01), count, np.float32)
    dev = to_dev(b, np.float32)
    args = [dev[k] for k in L.FIELDS]
    L.set_tuning(count, N, n, m, torch.float32, **_chunked(1, 1, True))
    try:
        eager = L.solve(*args, want_resid=True, refine=1)
        torch.cuda.synchronize()
        ref = {k: v.clone() for k, v in eager.items()}
        ws = L.Workspace()
        out = L.solve(*args, want_resid=True, refine=1, workspace=ws)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            L.solve(*args, want_resid=True, refine=1, workspace=ws, out=out)
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
        assert not ref["status"].any() and ref["resid"].max().item() <= RESID_TOL
        errs, res, _ = oracle_check_all(b, {k: v.cpu().numpy() for k, v in ref.items()}, as_f32=True)
        assert res.max() <= RESID_TOL and errs.max() <= FP32_ELEM_TOL
    finally:
        L.set_tuning(count, N, n, m, torch.float32, clear=True)


def test_leaf_building_sweep_status_bits():
    """At a shape whose chunk-1 sweep builds its leaves itself (n = 40,
    m = 8): an R_k of condition 1e7 sends only its instance to the FP64 redo
    (bit 8), which meets the oracle; with the fallback off an indefinite R_k
    sets bit 2 of only its instance."""
    N, n, m, count = 20, 40, 8, 4
    b = synth.gen_batch(lambda i: synth.gen_c1_like(N, n, m, [969, i], dt=0.01), count, np.float32)
    sched = _chunked(1, 1, True)
    ill = {k: v.copy() for k, v in b.items()}
    ill["R"][2, 7] = np.diag([1e-7] + [1.0] * (m - 1))
    say("[leaf-building sweep, ill-conditioned R]")
    out = _pinned(ill, np.float32, sched, want_resid=True, refine=1)
    assert out["status"][2] == 8 and not out["status"][[0, 1, 3]].any(), out["status"]
    errs, res = oracle_check(ill, out, 2, as_f32=True)
    say(f"  redone instance: elem err {errs}, resid gpu {out['resid'][2]:.2e} oracle {res:.2e}")
    assert out["resid"][2] <= RESID_TOL and res <= RESID_TOL
    bad = {k: v.copy() for k, v in b.items()}
    bad["R"][1, 3] = -100.0 * np.eye(m)
    say("[leaf-building sweep, indefinite R, fallback off]")
    out = _pinned(bad, np.float32, sched, fallback=False)
    assert out["status"][1] & 2 and not out["status"][1] & 8, out["status"]
    assert not out["status"][[0, 2, 3]].any(), out["status"]


def test_chunked_mappings_rejected():
    import torch
    import paper_2506_07823_amd as L
    with pytest.raises(L.LqrError):
        L.set_tuning(4, 10, 80, 12, torch.float32, engine="matrix-core", split=2, chunk=4, sweep=1)
    with pytest.raises(L.LqrError):
        L.set_tuning(4, 10, 12, 12, torch.float32, engine="wavefront", split=2, chunk=0, sweep=1)
    with pytest.raises(L.LqrError):
        L.set_tuning(4, 10, 12, 12, torch.float32, engine="wavefront", split=2, chunk=4, sweep=12)
    with pytest.raises(L.LqrError):
        L.set_tuning(4, 10, 12, 12, torch.float32, engine="wavefront", fused=2, fwd_seq=True)
