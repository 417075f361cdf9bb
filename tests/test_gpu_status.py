"""Per-instance status bits and argument errors of the C ABI on the GPU.

Failure conditions are planted in the host-side inputs (a NaN, an
indefinite R_k, an ill-conditioned R_k) or in the arguments (sizes, a short
workspace, a misaligned pointer); argument errors are rejected before any
launch."""
import ctypes

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


def _batch(count=3, N=10, n=6, m=3, dtype=np.float32):
    return synth.gen_batch(lambda i: synth.gen_rand(N, n, m, seed=[400, i]), count, dtype)


@pytest.mark.parametrize("method", ["scan", "plain"])
def test_indefinite_R_flags_only_that_instance(method):
    b = _batch(dtype=np.float64 if method == "plain" else np.float32)
    b["R"][1, 4] = -100.0 * np.eye(3)
    say(f"[status indefinite R {method}]")
    out = run(b, b["A"].dtype.type, method=method)
    assert out["status"][1] & 2
    assert out["status"][0] == 0 and out["status"][2] == 0


def test_nonfinite_input_flags_only_that_instance():
    b = _batch()
    b["c"][0, 3, 1] = np.nan
    say("[status nan input]")
    out = run(b, np.float32)
    assert out["status"][0] & 1
    assert out["status"][1] == 0 and out["status"][2] == 0


def test_ill_conditioned_R_takes_fp64_fallback():
    """cond(R_k) = 1e7 on generic data (B ~ 0.5 N(0, 1), the scaling at which
    FP32 records of the element cannot hold its C-tilde): the instance is
    marked and solved again whole in FP64 (bit 8 only), with the default one
    refinement sweep, and meets the oracle; the others keep clean status
    words."""
    b = _batch(N=12, n=8, m=4)
    b["R"][2, 5] = np.diag([1e-7, 1.0, 1.0, 1.0])
    say("[status ill-conditioned R fallback, generic scaling]")
    out = run(b, np.float32, want_resid=True)
    assert out["status"][2] == 8, out["status"]
    assert out["status"][0] == 0 and out["status"][1] == 0
    errs, res = oracle_check(b, out, 2, as_f32=True)
    say(f"  fallback instance: elem err {errs}, resid gpu {out['resid'][2]:.2e} oracle {res:.2e}")
    assert out["resid"][2] <= 1e-5 and res <= 1e-5
    assert max(errs) <= 1e-4
    for i in (0, 1):
        _, r = oracle_check(b, out, i, as_f32=True)
        assert r <= 1e-5


def test_ill_conditioned_R_fallback_configuration_scaling():
    """The same on data scaled like the configurations (B ~ N(0, 0.1))."""
    b = synth.gen_batch(lambda i: synth.gen_c1_like(12, 8, 4, [410, i]), 3, np.float32)
    b["R"][2, 5] = np.diag([1e-7, 1.0, 1.0, 1.0])
    say("[status ill-conditioned R fallback, configuration scaling]")
    out = run(b, np.float32, want_resid=True)
    assert out["status"][2] == 8, out["status"]
    assert out["status"][0] == 0 and out["status"][1] == 0
    errs, res = oracle_check(b, out, 2, as_f32=True)
    say(f"  fallback instance: elem err {errs}, resid gpu {out['resid'][2]:.2e} oracle {res:.2e}")
    assert out["resid"][2] <= 1e-5 and res <= 1e-5


def test_ill_conditioned_R_fallback_large_blocks():
    """Same on the matrix-core engine (order 70), generic scaling: the FP64
    redo of the large-block engine."""
    b = synth.gen_batch(lambda i: synth.gen_c1_like(8, 70, 12, [420, i]), 3, np.float32)
    b["R"][1, 3] = np.diag([1e-7] + [1.0] * 11)
    say("[status ill-conditioned R fallback, order 70]")
    out = run(b, np.float32, want_resid=True)
    assert out["status"][1] == 8, out["status"]
    assert out["status"][0] == 0 and out["status"][2] == 0
    errs, res = oracle_check(b, out, 1, as_f32=True)
    say(f"  fallback instance: elem err {errs}, resid gpu {out['resid'][1]:.2e} oracle {res:.2e}")
    assert out["resid"][1] <= 1e-5 and res <= 1e-5


def test_fallback_off_reports_the_failure():
    """With the fallback off an indefinite R_k sets the failure bit and a
    synchronous status check returns LQR_ENUMERIC."""
    import paper_2506_07823_amd as L
    b = _batch()
    b["R"][1, 4] = -100.0 * np.eye(3)
    say("[status fallback off, sync status]")
    out = run(b, np.float32, fallback=False)
    assert out["status"][1] & 2 and not out["status"][1] & 8
    dev = to_dev(b, np.float32)
    with pytest.raises(L.LqrError) as ei:
        L.solve(*[dev[k] for k in L.FIELDS], sync_status=True)
    assert ei.value.code == L.LQR_ENUMERIC
    clean = to_dev(_batch(), np.float32)
    r = L.solve(*[clean[k] for k in L.FIELDS], sync_status=True)
    assert not r["status"].any().item()


def _raw_call(dev, out, ws_bytes=None, batch=None, N=None, ptr_shift=0):
    import paper_2506_07823_amd as L
    bsz, Nn, n, m = L.dims_of(dev["A"], dev["B"])
    batch = bsz if batch is None else batch
    N = Nn if N is None else N
    o = L.default_opts()
    need = ctypes.c_size_t()
    assert L.lqr_workspace_size(L.handle(0), bsz, Nn, n, m, ctypes.byref(o), ctypes.byref(need)) == 0
    import torch
    wbytes = need.value if ws_bytes is None else ws_bytes
    ws = torch.empty(max(wbytes, 256), dtype=torch.uint8, device="cuda:0")
    ptrs = [dev[k].data_ptr() for k in L.FIELDS]
    ptrs[0] += ptr_shift
    return L.lqr_kkt_solve(L.handle(0), None, batch, N, n, m, *ptrs, out["x"].data_ptr(), out["u"].data_ptr(),
                           out["lam"].data_ptr(), out["status"].data_ptr(), ws.data_ptr(), wbytes,
                           ctypes.byref(o))


def test_argument_errors_launch_nothing():
    import torch
    import paper_2506_07823_amd as L
    b = _batch()
    dev = to_dev(b, np.float32)
    bsz, N, n, m = 3, 10, 6, 3
    out = {"x": torch.full((bsz, N + 1, n), 7.0, device="cuda:0"),
           "u": torch.full((bsz, N, m), 7.0, device="cuda:0"),
           "lam": torch.full((bsz, N + 1, n), 7.0, device="cuda:0"),
           "status": torch.full((bsz,), 99, dtype=torch.int32, device="cuda:0")}
    say("[errors] short workspace / bad sizes / misaligned")
    assert _raw_call(dev, out, ws_bytes=1024) == L.LQR_ENOMEM
    assert _raw_call(dev, out, batch=0) == L.LQR_EINVAL
    assert _raw_call(dev, out, N=0) == L.LQR_EINVAL
    assert _raw_call(dev, out, ptr_shift=2) == L.LQR_EINVAL
    torch.cuda.synchronize()
    assert (out["x"] == 7.0).all() and (out["status"] == 99).all()   # nothing ran
    assert _raw_call(dev, out) == L.LQR_OK
    torch.cuda.synchronize()
    assert (out["status"] == 0).all()
