"""Benchmark: batched LQR-KKT solves/s and p50/p99 latency on one MI355X.

Workload: whole-body-shaped LQR QPs, n = 36, m = 12, N = 100, a batch of
4096 independent seeded synthetic instances (inputs resident in HBM before
the timed region).  One step = one full hot-path pass over the batch: scan
elements, reverse associative scan (up-sweep + down-sweep), policy, forward
scan of the closed-loop maps, controls/costates, FP64 KKT residual, one
refinement sweep, and the FP64 residual of the returned solution (checked
<= 1e-5).  The comparison baseline ("plain") is the sequential FP64 Riccati
sweep on the same GPU and the same (FP64) problem data.

Prints ONE JSON line.  `python bench.py [--steps K] [--warmup W]`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LQR-KKT solves/s + p99 latency at rel KKT residual ≤1e-5: batched FP32 vs plain"
N_STAGES, NX, NU, BATCH = 100, 36, 12, 4096

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz.  The vector
# FP32 peak with packed-FP32 dual issue is twice that; this build compiles with
# packed FP32 disabled, so 78.6 TFLOP/s is the rate its VALU code can reach.
PEAK_FP32_VECTOR_PACKED = 157.3e12
PEAK_FP32_VECTOR = 256 * 4 * 16 * 2 * 2.4e9
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(L, dev, method, steps, warmup, want_timing, graph=False, refine=None):
    """Warm up, then time `steps` solves (each bracketed by events on the
    current stream).  graph=True captures one solve into a HIP graph and
    times its replays instead of eager launches."""
    import torch
    ws = L.Workspace()
    out = None
    for _ in range(warmup):
        out = L.solve(*[dev[k] for k in L.FIELDS], method=method, want_resid=True, out=out, workspace=ws,
                          refine=refine)
    torch.cuda.synchronize()
    g = None
    if graph:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            L.solve(*[dev[k] for k in L.FIELDS], method=method, want_resid=True, out=out, workspace=ws,
                    refine=refine)
        g.replay()
        torch.cuda.synchronize()
    if want_timing:
        L.kernel_timing(True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record()
        if g is not None:
            g.replay()
        else:
            out = L.solve(*[dev[k] for k in L.FIELDS], method=method, want_resid=True, out=out, workspace=ws,
                          refine=refine)
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    fams = None
    if want_timing:
        fams = L.kernel_report()
        L.kernel_timing(False)
    resid = out["resid"].max().item()
    status = int(out["status"].ne(0).sum().item())
    return wall, lat, fams, resid, status


def cpu_baseline(sample: int):
    import oracle
    import synth
    threads = min(os.cpu_count() or 1, 16)
    probs = synth.gen_batch(synth.gen_c3, sample, np.float32)
    probs = {k: v.astype(np.float64) for k, v in probs.items()}
    oracle.riccati_batch({k: v[:threads] for k, v in probs.items()}, nthreads=threads)  # warm
    t0 = time.perf_counter()
    _, _, _, st = oracle.riccati_batch(probs, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample} of the {BATCH} whole-body instances (FP32-rounded inputs in FP64), "
                      f"sequential Riccati in C on {threads} host threads, {dt:.2f} s wall",
            "failed": int((st != 0).sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of graph replays")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates the HBM byte "
                         "counters of a profiler against a known size) and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the batch-sharded multi-GPU form "
              "is described in DESIGN.md and not built", file=sys.stderr)
        sys.exit(2)

    import torch
    if a.copy_calib:
        nbytes = a.copy_calib << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": nbytes}), flush=True)
        return
    import paper_2506_07823_amd as L
    import synth

    log("[bench] generating inputs")
    host = synth.gen_batch(synth.gen_c3, BATCH, np.float32)
    dev = {k: torch.from_numpy(v).to("cuda:0") for k, v in host.items()}
    torch.cuda.synchronize()

    log("[bench] FP32 scan: timed graph replays")
    wall, lat, _, resid, bad = timed_steps(L, dev, "scan", a.steps, a.warmup, False, graph=not a.eager,
                                           refine=2)
    log("[bench] FP32 scan: kernel timing pass (eager, HIP events around every launch)")
    _, _, fams, _, _ = timed_steps(L, dev, "scan", max(3, a.steps // 5), 1, True, refine=2)
    value = BATCH * a.steps / wall
    result = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * wall / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "whole-body-shaped LQR-KKT, n=36 m=12 N=100, batch 4096, FP32 scan + "
                               "FP64-residual refinement (second sweep only above 1e-5)",
                   "batch": BATCH, "N": N_STAGES, "n": NX, "m": NU, "method": "scan",
                   "launch": "eager" if a.eager else "hipGraph replay"},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "max_rel_kkt_residual": resid, "instances_with_status": bad,
    }
    if fams:
        dom = max(fams, key=lambda f: fams[f]["ms"])
        d = fams[dom]
        avg_ms = d["ms"] / d["launches"]
        achieved = d["flops"] / (d["ms"] * 1e-3)
        result["roofline"] = {
            "kernel": dom, "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR, "traffic": None,
            "avg_launch_ms": avg_ms, "launches": d["launches"],
            "algorithmic_GBps": d["bytes"] / (d["ms"] * 1e-3) / 1e9,
            "peak_packed_fp32": PEAK_FP32_VECTOR_PACKED / 1e12,
        }
        steps_t = fams["clear"]["launches"] if "clear" in fams else 1
        result["kernel_ms_per_step"] = {f: v["ms"] / steps_t for f, v in fams.items()}
    if not a.no_plain:
        log("[bench] FP64 plain Riccati: timed steps")
        dev64 = {k: v.double() for k, v in dev.items()}
        del dev
        torch.cuda.empty_cache()
        pk = max(3, a.steps // 3)
        pwall, plat, _, presid, pbad = timed_steps(L, dev64, "plain", pk, 1, False, graph=not a.eager)
        result["plain"] = {"value": BATCH * pk / pwall, "unit": "solves/s", "dtype": "f64", "steps": pk,
                           "ms_per_step": 1e3 * pwall / pk, "p50_ms": float(np.percentile(plat, 50)),
                           "p99_ms": float(np.percentile(plat, 99)), "max_rel_kkt_residual": presid,
                           "instances_with_status": pbad}
        result["scan_over_plain"] = value / result["plain"]["value"]
    if not a.no_cpu:
        log("[bench] CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(a.cpu_sample)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
