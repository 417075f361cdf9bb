"""Helpers shared by the GPU tests: move seeded inputs to the device, run the
library, compare with the oracle."""
import sys

import numpy as np

import synth

FIELDS = synth.FIELDS


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
    return float(np.linalg.norm(np.asarray(a, float) - b) / max(np.linalg.norm(b), 1e-300))


def oracle_check(batch, out, b, as_f32=False):
    """Relative errors (x, u, lam) of instance b against the oracle, and the
    oracle-computed relative KKT residual of the GPU output."""
    import oracle
    prob = synth.instance(batch, b)
    if as_f32:
        prob = {k: v.astype(np.float32).astype(np.float64) for k, v in prob.items()}
    ref = oracle.riccati(prob)
    errs = tuple(rel(out[f][b], ref[f]) for f in ("x", "u", "lam"))
    res = oracle.rel_kkt_residual(prob, out["x"][b].astype(np.float64), out["u"][b].astype(np.float64),
                                  out["lam"][b].astype(np.float64))
    return errs, res
