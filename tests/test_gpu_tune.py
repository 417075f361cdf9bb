"""Autotuner and pinned mappings: every candidate mapping of a shape meets
the same bars (FP64 relative error <= 1e-9 against the oracle), the
vector-pass forms give identical bits, and the tuned choice is used by the
following solves of that shape."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import oracle_check, run, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401


SHAPE = (12, 40, 12)   # both engines can take it


def _batch(count, dtype):
    N, n, m = SHAPE
    return synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[800, i]), count, dtype)


@pytest.mark.parametrize("engine,fused,grid,extra", [
    ("wavefront", False, 0, {}), ("wavefront", True, 0, {}), ("wavefront", 2, 0, {}),
    ("wavefront", False, 0, {"split": 1}), ("wavefront", False, 0, {"split": 2, "chunk": 4, "sweep": 3}),
    ("wavefront", False, 0, {"split": 2, "chunk": 1, "sweep": 1, "fwd_seq": True}),
    ("wavefront", False, 0, {"fwd_seq": True}),
    ("matrix-core", False, 256, {}), ("matrix-core", True, 512, {}), ("matrix-core", False, 512, {"fwd_seq": True})])
def test_every_mapping_meets_the_bar(engine, fused, grid, extra):
    import torch
    import paper_2506_07823_amd as L
    N, n, m = SHAPE
    b = _batch(3, np.float64)
    say(f"[mapping {engine} fused={fused} grid={grid} {extra}]")
    L.set_tuning(3, N, n, m, torch.float64, engine=engine, fused=fused, big_grid=grid, **extra)
    try:
        out = run(b, np.float64)
    finally:
        L.set_tuning(3, N, n, m, torch.float64, clear=True)
    assert not out["status"].any()
    for i in range(3):
        errs, res = oracle_check(b, out, i)
        assert max(errs) <= 1e-9 and res <= 1e-11, (i, errs)


def test_vector_pass_forms_bitwise_equal():
    import torch
    import paper_2506_07823_amd as L
    N, n, m = SHAPE
    b = _batch(4, np.float32)
    outs = []
    for fused in (0, 1, 2):
        L.set_tuning(4, N, n, m, torch.float32, engine="wavefront", fused=fused)
        outs.append(run(b, np.float32, refine=2, want_resid=True))
    L.set_tuning(4, N, n, m, torch.float32, clear=True)
    for o in outs[1:]:
        for f in ("x", "u", "lam", "resid"):
            assert np.array_equal(outs[0][f], o[f]), f


def test_autotune_picks_and_pins_a_mapping():
    import torch
    import paper_2506_07823_amd as L
    N, n, m = SHAPE
    b = _batch(64, np.float32)
    dev = to_dev(b, np.float32)
    best = L.autotune(*[dev[k] for k in synth.FIELDS], refine=2, reps=2)
    say(f"[autotune] N={N} n={n} m={m} batch=64 -> {best}")
    assert best["engine"] in ("wavefront", "matrix-core") and best["ms"] > 0
    out = L.solve(*[dev[k] for k in synth.FIELDS], refine=2, want_resid=True)
    torch.cuda.synchronize()
    assert not out["status"].any()
    assert out["resid"].max().item() <= 1e-5
    L.set_tuning(64, N, n, m, torch.float32, clear=True)


def test_set_tuning_rejects_bad_mappings():
    import paper_2506_07823_amd as L
    with pytest.raises(L.LqrError):
        L.set_tuning(1, 10, 100, 10, engine="wavefront")   # order 100 has no wavefront class
    with pytest.raises(L.LqrError):
        L.set_tuning(1, 10, 10, 10, engine="matrix-core", big_grid=-1)
    with pytest.raises(L.LqrError):
        L.set_tuning(1, 10, 10, 10, engine="matrix-core", fused=2)   # one-launch form: wavefront engine only
    with pytest.raises(L.LqrError):
        L.set_tuning(1, 10, 100, 10, fused=2)
    with pytest.raises(L.LqrError):
        L.set_tuning(1, 10, 10, 10, fused=3)


def test_tuning_cache_round_trip(tmp_path):
    """The autotuned choice is kept per shape bucket, written to a cache file
    and read back (entries of this device's architecture only)."""
    import torch
    import paper_2506_07823_amd as L
    N, n, m = SHAPE
    b = _batch(16, np.float32)
    dev = to_dev(b, np.float32)
    best = L.autotune(*[dev[k] for k in synth.FIELDS], reps=1)
    path = str(tmp_path / "tune.txt")
    L.save_tuning(path)
    lines = open(path).read().splitlines()
    say(f"[tuning cache] {best} -> {lines}")
    assert any(line.startswith("lqr-tune-1 gfx950 0 %d %d " % (n, m)) for line in lines)
    with open(path, "a") as f:
        f.write("lqr-tune-1 gfx000 0 4 2 16 1 1 0 0 0 0 0 0\n")   # another architecture: kept, not loaded
    L.set_tuning(16, N, n, m, torch.float32, clear=True)
    assert L.load_tuning(path) >= 1
    L.save_tuning(path)
    assert any(line.startswith("lqr-tune-1 gfx000 ") for line in open(path).read().splitlines())
    out = L.solve(*[dev[k] for k in synth.FIELDS], want_resid=True)
    torch.cuda.synchronize()
    assert not out["status"].any() and out["resid"].max().item() <= 1e-5
    L.set_tuning(16, N, n, m, torch.float32, clear=True)
