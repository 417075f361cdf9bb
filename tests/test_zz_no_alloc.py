"""The no-allocation entry point (lqr_kkt_solve_noalloc: workspace in a
fixed per-GPU array of the library) gives the bits of lqr_kkt_solve with a
caller workspace, on two calls in a row (the second smaller, so the array
holds the first call's leftovers), and refuses a problem larger than its
array without launching anything."""
import ctypes

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
    import paper_2506_07823_amd  # noqa: F401


def _outputs(batch, N, n, m, dtype):
    import torch
    return {"x": torch.full((batch, N + 1, n), 7.0, dtype=dtype, device="cuda:0"),
            "u": torch.full((batch, N, m), 7.0, dtype=dtype, device="cuda:0"),
            "lam": torch.full((batch, N + 1, n), 7.0, dtype=dtype, device="cuda:0"),
            "status": torch.full((batch,), 99, dtype=torch.int32, device="cuda:0"),
            "resid": torch.zeros((batch,), dtype=torch.float64, device="cuda:0")}


def _noalloc(L, dev, out, dtype):
    import torch
    batch, N, n, m = L.dims_of(dev["A"], dev["B"])
    o = L.default_opts(dtype)
    o.resid_out = out["resid"].data_ptr()
    s = torch.cuda.current_stream().cuda_stream
    return L.lqr_kkt_solve_noalloc(L.handle(0), s, batch, N, n, m, *[dev[k].data_ptr() for k in L.FIELDS],
                                   out["x"].data_ptr(), out["u"].data_ptr(), out["lam"].data_ptr(),
                                   out["status"].data_ptr(), ctypes.byref(o))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_no_alloc_equals_workspace_entry_point(dtype):
    import torch
    import paper_2506_07823_amd as L
    npdt = np.float32 if dtype == "f32" else np.float64
    tdt = torch.float32 if dtype == "f32" else torch.float64
    assert L.lqr_noalloc_workspace_bytes() == 64 << 20
    cases = [(6, 50, 12, 12, lambda i: synth.gen_c2(50, i)), (2, 25, 12, 12, lambda i: synth.gen_c2(25, i))]
    for count, N, n, m, gen in cases:
        say(f"[no-alloc {dtype}] batch={count} N={N} n={n} m={m}")
        b = synth.gen_batch(gen, count, npdt)
        dev = to_dev(b, npdt)
        ref = L.solve(*[dev[k] for k in L.FIELDS], want_resid=True)
        torch.cuda.synchronize()
        out = _outputs(count, N, n, m, tdt)
        rc = _noalloc(L, dev, out, tdt)
        assert rc == L.LQR_OK, L.lqr_last_error()
        torch.cuda.synchronize()
        assert not out["status"].any().item()
        for k in ("x", "u", "lam", "status", "resid"):
            assert torch.equal(out[k], ref[k]), k


def test_no_alloc_refuses_a_problem_beyond_its_array():
    import torch
    import paper_2506_07823_amd as L
    count, N, n, m = 64, 100, 36, 12
    say(f"[no-alloc too large] batch={count} N={N} n={n} m={m}")
    b = synth.gen_batch(synth.gen_c3, count, np.float32)
    dev = to_dev(b, np.float32)
    out = _outputs(count, N, n, m, torch.float32)
    assert _noalloc(L, dev, out, torch.float32) == L.LQR_ENOMEM
    assert b"no-allocation" in L.lqr_last_error()
    torch.cuda.synchronize()
    assert (out["status"] == 99).all().item() and (out["x"] == 7.0).all().item()   # nothing ran
