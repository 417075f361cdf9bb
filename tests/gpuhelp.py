"""Helpers shared by the GPU tests: move seeded inputs to the device, run the
library, compare with the oracle element by element."""
import os
import sys

import numpy as np

import synth

FIELDS = synth.FIELDS
OUTS = ("x", "u", "lam")

# Element-wise gates (see elem_err): FP64 paths against the FP64 oracle, and
# the FP32 path (FP32 storage of inputs and results, one FP64-residual
# refinement sweep) against the oracle solved on the same FP32-rounded
# inputs.  After the sweep the solve error is below the FP32 rounding of the
# stored result (6e-8 relative per entry) times the conditioning of these
# KKT systems (up to ~10 at the scale of elem_err): measured at most 6.3e-7
# over every FP32 test instance; the gate is that times ~8.
FP64_ELEM_TOL = 1e-9
FP32_ELEM_TOL = 5e-6
RESID_TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(batch, dtype):
    import torch
    td = torch.float32 if dtype == np.float32 else torch.float64
    return {k: torch.from_numpy(np.ascontiguousarray(batch[k], dtype=dtype)).to("cuda:0", td) for k in FIELDS}


def run(batch, dtype, **kw):
    import torch
    import paper_2506_07823_amd as L
    dev = to_dev(batch, dtype)
    out = L.solve(*[dev[k] for k in FIELDS], **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def rel(a, b):
    """Normwise relative error (reported, not a gate)."""
    return float(np.linalg.norm(np.asarray(a, float) - b) / max(np.linalg.norm(b), 1e-300))


def elem_err(a, ref):
    """max_i |a_i - ref_i| / (|ref_i| + max_j |ref_j|) over one output block:
    an element-wise relative error whose absolute floor is the block's
    largest entry (so a wrong small entry is caught at the scale of the
    block, not hidden under its 2-norm)."""
    a = np.asarray(a, float)
    ref = np.asarray(ref, float)
    scale = np.abs(ref) + max(float(np.abs(ref).max()), 1e-300)
    return float(np.max(np.abs(a - ref) / scale))


def elem_err_batch(a, ref):
    """elem_err of every instance (leading axis) of a batched block."""
    a = np.asarray(a, float).reshape(a.shape[0], -1)
    ref = np.asarray(ref, float).reshape(ref.shape[0], -1)
    top = np.maximum(np.abs(ref).max(axis=1, keepdims=True), 1e-300)
    return np.max(np.abs(a - ref) / (np.abs(ref) + top), axis=1)


def as_oracle_input(batch, as_f32):
    if as_f32:
        return {k: np.asarray(v).astype(np.float32).astype(np.float64) for k, v in batch.items()}
    return {k: np.asarray(v, np.float64) for k, v in batch.items()}


def oracle_check(batch, out, b, as_f32=False):
    """Element-wise errors (x, u, lam) of instance b against the oracle, and
    the oracle-computed relative KKT residual of the GPU output."""
    import oracle
    prob = synth.instance(batch, b)
    if as_f32:
        prob = {k: v.astype(np.float32).astype(np.float64) for k, v in prob.items()}
    ref = oracle.riccati(prob)
    errs = tuple(elem_err(out[f][b], ref[f]) for f in OUTS)
    res = oracle.rel_kkt_residual(prob, out["x"][b].astype(np.float64), out["u"][b].astype(np.float64),
                                  out["lam"][b].astype(np.float64))
    return errs, res


def oracle_check_all(batch, out, as_f32=False):
    """Every instance of a batch against the oracle (its batched solve on the
    host threads): per-instance element-wise errors of x, u, lam (array
    [batch, 3]), the oracle-computed relative KKT residual of each GPU
    solution, and the oracle's status words."""
    import oracle
    probs = as_oracle_input(batch, as_f32)
    threads = min(os.cpu_count() or 1, 16)
    x, u, lam, st = oracle.riccati_batch(probs, nthreads=threads)
    errs = np.stack([elem_err_batch(out["x"], x), elem_err_batch(out["u"], u), elem_err_batch(out["lam"], lam)],
                    axis=1)
    count = probs["x0"].shape[0]
    res = np.array([oracle.rel_kkt_residual({k: v[b] for k, v in probs.items()}, out["x"][b].astype(np.float64),
                                            out["u"][b].astype(np.float64), out["lam"][b].astype(np.float64))
                    for b in range(count)])
    return errs, res, st


def describe(name, errs, res):
    say(f"  {name}: element-wise err max {errs.max():.2e} (x {errs[:, 0].max():.2e}, u {errs[:, 1].max():.2e}, "
        f"lam {errs[:, 2].max():.2e}), p50 {np.median(errs.max(axis=1)):.2e}; oracle resid max {res.max():.2e} "
        f"p50 {np.median(res):.2e}")
