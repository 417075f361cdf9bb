"""Benchmark: batched LQR-KKT solves/s and p50/p99 latency on one MI355X.

Workload: whole-body-shaped LQR QPs, n = 36, m = 12, N = 100, a batch of
4096 independent seeded synthetic instances (inputs resident in HBM before
the timed region).  One step = one full hot-path pass over the batch: scan
elements, reverse associative scan (up-sweep + down-sweep), policy, forward
scan of the closed-loop maps, controls/costates, FP64 KKT residual,
refinement sweeps for the instances above 1e-5 (at most two), and the FP64
residual of the returned solution (checked <= 1e-5).  The mapping is
autotuned first.  The comparison baseline ("plain") is the sequential FP64
Riccati sweep on the same GPU and the same (FP64) problem data.

A second object ("multi_robot") measures the centralized multi-robot shape,
n = m = 192, N = 50, batch 64, on the large-block (matrix-core) engine the
same way, and "serving" runs a Poisson stream of mixed requests (60 %
SRBD-shaped, 30 % whole-body-shaped, 10 % multi-robot) through the
continuous-batching loop at 70 % of its measured capacity (p50/p99 latency
from arrival, host-to-device copies included).  "latency" times single
SRBD-shaped solves (n = m = 12, batch 1, N = 25 .. 200): FP32 scan against
the FP64 plain Riccati sweep, both as graph replays; "batch_sweep" runs the
whole-body workload at batches 16 .. 1024 (scan and plain solves/s).

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

# MI355X published peaks.  FP32 vector: 157.3 TFLOP/s (256 CUs x 4 SIMD x 16
# lanes x 2 flops (FMA) x 2.4 GHz x 2 for packed-FP32 dual issue).  The
# library is compiled with packed FP32 disabled, so the rate its VALU code can
# reach is half of that, 78.6 TFLOP/s; both are reported.
PEAK_FP32_VECTOR = 157.3e12
PEAK_FP32_VECTOR_NONPACKED = 256 * 4 * 16 * 2 * 2.4e9
PEAK_FP64_VECTOR = 78.6e12
PEAK_HBM = 8.0e12
# dense FP32 matrix-core peak (MFMA), the bound of the large-block engine
PEAK_FP32_MFMA = 157.3e12
MR_BATCH = 64
LAT_REPLAYS = 200   # graph replays of the dedicated p50/p99 loops

# HBM bytes per launch of the whole-body dominant kernel from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs, calibrated against a copy of known size;
# valid only for the kernel and launch sources they were taken on (hash of
# every source file of the library)
TRAFFIC = {"kernel": "chunk_mid", "src_hash": "a5cc678d0e1ffec9", "bytes_per_launch": 9.311e9,
           "note": "rocprofv3 FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 (factors from a 1 GiB device copy), "
                   "4 eager one-stream dispatches of k_chunk_mid_elem (leaf-building sweep) at batch 4096, "
                   "chunk 1: 7.077 + 2.234 GB per launch"}


def kernel_src_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_07823_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


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


def host_info() -> dict:
    """Host CPU facts for the oracle baseline: model, core counts, compiler."""
    import platform
    import subprocess
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
    except (OSError, ValueError):
        nproc = None
    try:
        gcc = subprocess.run(["gcc", "--version"], capture_output=True, text=True).stdout.splitlines()[0]
    except (OSError, IndexError):
        gcc = None
    return {"cpu_model": model, "nproc": nproc, "os_cpu_count": os.cpu_count(),
            "sched_affinity": len(os.sched_getaffinity(0)), "compiler": gcc}


def cpu_baseline(gen, sample: int, batch: int, what: str):
    """The oracle (sequential FP64 Riccati in C) built for this host with
    -march=native, one instance per task over all the host cores this process
    may use (at most 16, the CPU share of one GPU on the benchmark machines),
    on a sample of the workload's instances."""
    import tempfile
    import oracle
    import synth
    info = host_info()
    threads = max(1, min(info["sched_affinity"] or 1, 16))
    tmpdir = tempfile.mkdtemp(prefix="lqr_oracle_")
    lib = oracle.load_library(oracle.build_native(os.path.join(tmpdir, "liblqr_oracle_native.so")))
    old = oracle.use_library(lib)
    try:
        probs = synth.gen_batch(gen, sample, np.float32)
        probs = {k: v.astype(np.float64) for k, v in probs.items()}
        oracle.riccati_batch({k: v[:1] for k, v in probs.items()}, nthreads=1)  # warm
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            _, _, _, st = oracle.riccati_batch(probs, nthreads=threads)
            runs.append(time.perf_counter() - t0)
        dt = float(np.median(runs))
    finally:
        oracle.use_library(old)
    return {"value": sample / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample} of the {batch} {what} instances (FP32-rounded inputs in FP64), sequential Riccati "
                      f"in C (gcc -O3 -march=native) on {threads} host threads, median of 3 runs, {dt:.2f} s wall",
            "failed": int((st != 0).sum()), "host": info}


def roofline_of(fams, bound, peak, unit):
    """Dominant kernel family of a timing pass: algorithmic work (the
    method's per-unit cost model) / measured time."""
    dom = max(fams, key=lambda f: fams[f]["ms"])
    d = fams[dom]
    achieved = d["flops"] / (d["ms"] * 1e-3)
    return {"kernel": dom, "bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": unit,
            "frac": achieved / peak, "traffic": None, "avg_launch_ms": d["ms"] / d["launches"],
            "launches": d["launches"], "flops_per_launch": d["flops"] / d["launches"],
            "algorithmic_bytes_per_launch": d["bytes"] / d["launches"],
            "algorithmic_GBps": d["bytes"] / (d["ms"] * 1e-3) / 1e9,
            "achieved_executed_form_count": d["flops_min"] / (d["ms"] * 1e-3) / 1e12}


def replay_latency(L, dev, method, refine, replays):
    """p50/p99 of `replays` graph replays of one solve (each bracketed by
    events), outside the timed region."""
    import torch
    ws = L.Workspace()
    out = L.solve(*[dev[k] for k in L.FIELDS], method=method, want_resid=True, workspace=ws, refine=refine)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        L.solve(*[dev[k] for k in L.FIELDS], method=method, want_resid=True, out=out, workspace=ws, refine=refine)
    g.replay()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(replays)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(replays)]
    for i in range(replays):
        starts[i].record()
        g.replay()
        ends[i].record()
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    return {"replays": replays, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max())}


def residual_profile(L, dev, refine_tol):
    """The raw FP32 scan (no refinement sweep) on the same inputs: the
    distribution of its relative KKT residual and how many instances the
    refinement sweep takes (those above the tolerance)."""
    import torch
    out = L.solve(*[dev[k] for k in L.FIELDS], refine=0, want_resid=True)
    torch.cuda.synchronize()
    r = out["resid"].cpu().numpy()
    return {"raw_resid_p50": float(np.percentile(r, 50)), "raw_resid_p99": float(np.percentile(r, 99)),
            "raw_resid_max": float(r.max()), "refine_tol": refine_tol,
            "instances_refined": int((r > refine_tol).sum()), "instances": int(r.size)}


def measure(L, gen, batch, steps, warmup, eager, refine, plain, label, tune=True, pin=None, replays=LAT_REPLAYS):
    """Timed FP32 scan (graph replays) + kernel-timing pass + p50/p99 of a
    dedicated replay loop + optional FP64 plain comparison on one workload;
    returns the numbers and the timing families of the scan."""
    import torch
    import synth
    log(f"[bench] {label}: generating inputs")
    host = synth.gen_batch(gen, batch, np.float32)
    dev = {k: torch.from_numpy(v).to("cuda:0") for k, v in host.items()}
    del host
    torch.cuda.synchronize()
    N_, n_, m_ = dev["B"].shape[1:]
    mapping = "default"
    if pin:
        L.set_tuning(batch, N_, n_, m_, torch.float32, **pin)
        mapping = dict(pin)
    elif tune:
        log(f"[bench] {label}: autotuning the mapping")
        mapping = L.autotune(*[dev[k] for k in L.FIELDS], refine=refine, reps=2)
        log(f"[bench] {label}: mapping {mapping}")
    log(f"[bench] {label}: FP32 scan, timed {'eager launches' if eager else 'graph replays'}")
    wall, _, _, resid, bad = timed_steps(L, dev, "scan", steps, warmup, False, graph=not eager, refine=refine)
    log(f"[bench] {label}: FP32 scan, {replays} graph replays for p50/p99")
    lat = replay_latency(L, dev, "scan", refine, replays)
    log(f"[bench] {label}: FP32 scan, kernel timing pass (eager, HIP events around every launch)")
    _, _, fams, _, _ = timed_steps(L, dev, "scan", max(3, steps // 5), 1, True, refine=refine)
    fams_split = None
    if isinstance(mapping, dict) and mapping.get("streams", 0) > 1:
        # The batch split over streams overlaps the parts' launches, so a
        # launch's event-to-event time also holds other parts' GPU time.
        # The kernels' own rates come from a second pass of the same mapping
        # on one stream (each launch then has the GPU to itself).
        fams_split = fams
        one = mapping_kwargs(mapping)
        one["streams"] = 0
        log(f"[bench] {label}: FP32 scan, kernel timing pass of the same mapping on one stream")
        L.set_tuning(batch, N_, n_, m_, torch.float32, **one)
        _, _, fams, _, _ = timed_steps(L, dev, "scan", max(3, steps // 5), 1, True, refine=refine)
        L.set_tuning(batch, N_, n_, m_, torch.float32, **mapping_kwargs(mapping))
    tol = L.default_opts().refine_tol
    r = {"value": batch * steps / wall, "unit": "solves/s", "steps": steps, "ms_per_step": 1e3 * wall / steps,
         "p50_ms": lat["p50_ms"], "p99_ms": lat["p99_ms"], "latency_replays": replays,
         "max_rel_kkt_residual": resid, "instances_with_status": bad,
         "refinement": {"sweeps": refine, **residual_profile(L, dev, tol)}}
    steps_t = fams["clear"]["launches"] if "clear" in fams else 1
    r["kernel_ms_per_step"] = {f: v["ms"] / steps_t for f, v in fams.items()}
    if fams_split is not None:
        st = mapping["streams"]
        r["kernel_timing"] = "eager pass of the same mapping on one stream (kernel_ms_per_step, roofline)"
        r["kernel_ms_per_step_overlapped"] = {
            "note": f"eager pass with the batch in {st} parts on {st} streams: event-to-event time of each part's "
                    f"launches, summed over the parts, which overlap one another",
            **{f: v["ms"] / steps_t for f, v in fams_split.items()}}
    r["mapping"] = mapping
    # useful work: the plain sequential Riccati's count of the same solves
    plain_f = N_ * (4 * n_ ** 3 + 6 * n_ ** 2 * m_ + 4 * n_ * m_ ** 2 + m_ ** 3 / 3)
    scan_f = sum(v["flops"] for v in fams.values()) / steps_t
    r["work"] = {"plain_count_flops_per_solve": plain_f, "scan_count_flops_per_solve": scan_f / batch,
                 "useful_TFLOPs": r["value"] * plain_f / 1e12,
                 "executed_TFLOPs": scan_f / (r["ms_per_step"] * 1e-3) / 1e12}
    if plain:
        log(f"[bench] {label}: FP64 plain Riccati, timed steps")
        dev64 = {k: v.double() for k, v in dev.items()}
        del dev
        torch.cuda.empty_cache()
        pk = max(3, steps // 3)
        pwall, _, _, presid, pbad = timed_steps(L, dev64, "plain", pk, 1, False, graph=not eager)
        plat = replay_latency(L, dev64, "plain", 0, max(20, replays // 2))
        r["plain"] = {"value": batch * pk / pwall, "unit": "solves/s", "dtype": "f64", "steps": pk,
                      "ms_per_step": 1e3 * pwall / pk, "p50_ms": plat["p50_ms"], "p99_ms": plat["p99_ms"],
                      "latency_replays": plat["replays"], "max_rel_kkt_residual": presid,
                      "instances_with_status": pbad,
                      "useful_TFLOPs": batch * pk / pwall * plain_f / 1e12,
                      "frac_of_fp64_peak": batch * pk / pwall * plain_f / PEAK_FP64_VECTOR}
        r["scan_over_plain"] = r["value"] / r["plain"]["value"]
        del dev64
    else:
        del dev
    torch.cuda.empty_cache()
    return r, fams


def mapping_kwargs(mapping):
    """set_tuning keyword arguments of an autotuned (or pinned) mapping."""
    kw = {k: v for k, v in mapping.items() if k != "ms"}
    if "fwd_seq" in kw:
        kw["fwd_seq"] = bool(kw["fwd_seq"])
    return kw


def fused_steps(L, dev, N, n, m, batch, steps, **mapping):
    """timed_steps of the FP32 scan with a wavefront-engine mapping pinned
    for this shape (default: the one-launch form, the whole solve in one
    kernel per instance), then the pin cleared."""
    import torch
    mapping = mapping or {"fused": 2}
    L.set_tuning(batch, N, n, m, torch.float32, engine="wavefront", **mapping)
    try:
        return timed_steps(L, dev, "scan", steps, 2, False, graph=True, refine=1)
    finally:
        L.set_tuning(batch, N, n, m, torch.float32, clear=True)


def latency_leg(L, steps: int = 50):
    """Single-solve latency of the SRBD-shaped case (n = m = 12, one
    instance) at every horizon: graph replays of the FP32 scan (with its
    refinement) against the FP64 plain Riccati sweep, p50/p99 over `steps`
    replays each.  The scan's O(log N) depth against N dependent steps."""
    import torch
    import synth
    out = {}
    for N in synth.C2_HORIZONS:
        host = synth.gen_batch(lambda i: synth.gen_c2(N, i), 1, np.float32)
        dev = {k: torch.from_numpy(v).to("cuda:0") for k, v in host.items()}
        _, lat, _, resid, bad = timed_steps(L, dev, "scan", steps, 3, False, graph=True, refine=1)
        _, flat, _, fresid, fbad = fused_steps(L, dev, N, 12, 12, 1, steps)
        dev64 = {k: v.double() for k, v in dev.items()}
        _, plat, _, presid, pbad = timed_steps(L, dev64, "plain", steps, 3, False, graph=True)
        out[f"N{N}"] = {"scan_p50_ms": float(np.percentile(lat, 50)), "scan_p99_ms": float(np.percentile(lat, 99)),
                        "one_launch_p50_ms": float(np.percentile(flat, 50)),
                        "one_launch_p99_ms": float(np.percentile(flat, 99)),
                        "plain_p50_ms": float(np.percentile(plat, 50)),
                        "plain_p99_ms": float(np.percentile(plat, 99)),
                        "scan_rel_kkt_residual": max(resid, fresid), "plain_rel_kkt_residual": presid,
                        "instances_with_status": bad + fbad + pbad}
        log(f"[bench] latency N={N}: scan p50 {out[f'N{N}']['scan_p50_ms']:.3f} ms, "
            f"one launch p50 {out[f'N{N}']['one_launch_p50_ms']:.3f} ms, "
            f"plain p50 {out[f'N{N}']['plain_p50_ms']:.3f} ms")
    out["workload"] = ("SRBD-shaped single solve (n=m=12, batch 1), hipGraph replays, FP32 scan + refinement "
                       "(level-by-level launches, and the one-launch form) vs FP64 plain")
    return out


def batch_sweep_leg(L, batches=(16, 64, 256, 1024), steps: int = 10):
    """Whole-body workload at smaller batches (default mapping, graph
    replays): solves/s of the FP32 scan and of the FP64 plain sweep, to show
    where the scan's depth outweighs its extra arithmetic."""
    import torch
    import synth
    host = synth.gen_batch(synth.gen_c3, max(batches), np.float32)
    rows = {}
    for B in batches:
        dev = {k: torch.from_numpy(np.ascontiguousarray(v[:B])).to("cuda:0") for k, v in host.items()}
        wall, lat, _, resid, bad = timed_steps(L, dev, "scan", steps, 2, False, graph=True, refine=1)
        fwall, flat, _, fresid, fbad = fused_steps(L, dev, 100, 36, 12, B, steps)
        swall, slat, _, sresid, sbad = fused_steps(L, dev, 100, 36, 12, B, steps, fused=0, split=True)
        qwall, qlat, _, qresid, qbad = fused_steps(L, dev, 100, 36, 12, B, steps, fused=0, split=2, chunk=1,
                                                   sweep=1, fwd_seq=True)
        mapping = L.autotune(*[dev[k] for k in L.FIELDS], refine=1, reps=2)
        twall, tlat, _, tresid, tbad = timed_steps(L, dev, "scan", steps, 2, False, graph=True, refine=1)
        L.set_tuning(B, 100, 36, 12, torch.float32, clear=True)
        dev64 = {k: v.double() for k, v in dev.items()}
        pwall, plat, _, presid, pbad = timed_steps(L, dev64, "plain", steps, 2, False, graph=True)
        rows[f"B{B}"] = {"scan_solves_per_s": B * steps / wall, "one_launch_solves_per_s": B * steps / fwall,
                         "split_solves_per_s": B * steps / swall, "sequential_solves_per_s": B * steps / qwall,
                         "tuned_solves_per_s": B * steps / twall, "tuned_mapping": mapping,
                         "plain_solves_per_s": B * steps / pwall,
                         "scan_p50_ms": float(np.percentile(lat, 50)), "one_launch_p50_ms": float(np.percentile(flat, 50)),
                         "split_p50_ms": float(np.percentile(slat, 50)),
                         "sequential_p50_ms": float(np.percentile(qlat, 50)),
                         "tuned_p50_ms": float(np.percentile(tlat, 50)),
                         "plain_p50_ms": float(np.percentile(plat, 50)),
                         "scan_rel_kkt_residual": max(resid, fresid, sresid, qresid, tresid),
                         "instances_with_status": bad + fbad + sbad + qbad + tbad + pbad}
        log(f"[bench] batch {B}: scan {rows[f'B{B}']['scan_solves_per_s']:.0f}/s, "
            f"one launch {rows[f'B{B}']['one_launch_solves_per_s']:.0f}/s, "
            f"split {rows[f'B{B}']['split_solves_per_s']:.0f}/s, "
            f"chunk 1 {rows[f'B{B}']['sequential_solves_per_s']:.0f}/s, "
            f"autotuned {rows[f'B{B}']['tuned_solves_per_s']:.0f}/s, "
            f"plain {rows[f'B{B}']['plain_solves_per_s']:.0f}/s")
        del dev, dev64
    rows["workload"] = ("whole-body-shaped (n=36, m=12, N=100), hipGraph replays: default mapping (level-by-level "
                        "launches, balanced tree), the one-launch form, the split schedule (tree over 64 elements, "
                        "sequential sweep over 37), the chunked schedule with chunk 1 and sequential vector passes, the "
                        "mapping the autotuner picks for the batch (tuned_mapping), and the FP64 plain sweep")
    return rows


def resolve_leg(L, batch=BATCH, replays=20):
    """Whole-body batch: a full solve, then lqr_kkt_resolve with new
    (x0, c, q, r) (the factors cached in the workspace reused), both as graph
    replays: the real-time-iteration re-solve against the full solve."""
    import torch
    import synth
    host = synth.gen_batch(synth.gen_c3, batch, np.float32)
    dev = {k: torch.from_numpy(v).to("cuda:0") for k, v in host.items()}
    del host
    ws = L.Workspace()
    out = L.solve(*[dev[k] for k in L.FIELDS], workspace=ws, want_resid=True, refine=1)
    torch.cuda.synchronize()
    dev2 = dict(dev)
    g = torch.Generator(device="cpu").manual_seed(11)
    for f, sd in (("x0", 1e-2), ("q", 1e-1)):
        dev2[f] = dev[f] + (sd * torch.randn(dev[f].shape, generator=g)).to("cuda:0")
    L.resolve(*[dev2[k] for k in L.FIELDS], out=out, workspace=ws, want_resid=True, refine=1)
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        L.resolve(*[dev2[k] for k in L.FIELDS], out=out, workspace=ws, want_resid=True, refine=1)
    gs = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gs):
        L.solve(*[dev[k] for k in L.FIELDS], workspace=ws, want_resid=True, refine=1, out=out)
    times = {}
    for name, gg in (("solve", gs), ("resolve", gr)):
        gg.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(replays):
            gg.replay()
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / replays
    gr.replay()
    torch.cuda.synchronize()
    res = {"workload": f"whole-body-shaped, batch {batch}: full solve, then new x0 and q with the same matrices",
           "solve_ms": times["solve"], "resolve_ms": times["resolve"], "speedup": times["solve"] / times["resolve"],
           "resolve_solves_per_s": batch / times["resolve"] * 1e3,
           "resolve_max_rel_kkt_residual": out["resid"].max().item(),
           "instances_with_status": int(out["status"].ne(0).sum().item())}
    log(f"[bench] resolve: solve {times['solve']:.2f} ms, resolve {times['resolve']:.2f} ms")
    return res


def sqp_leg(L, batch=1024, iters=10):
    """Batched SQP iterations (linearize, QP blocks, scan solve, parallel
    filter line search, update) on the synthetic bilinear model at the
    whole-body shape with 24 constraints; ms per iteration and the step
    lengths taken."""
    import torch
    import synth
    N, n, m, nc = 100, 36, 12, 24
    mb = synth.gen_bilinear_batch(batch, N, n, m, nc, [7], 0.05, dtype=np.float32)
    md = {k: torch.from_numpy(np.ascontiguousarray(mb[k])).to("cuda:0") for k in L.MODEL_FIELDS}
    md["gamma"] = mb["gamma"]

    def start():
        X = torch.from_numpy(np.ascontiguousarray(np.repeat(mb["xhat0"][:, None, :], N + 1, axis=1))).to("cuda:0")
        return X, torch.zeros((batch, N, m), device="cuda:0"), torch.zeros((batch, N + 1, n), device="cuda:0")

    # the mapping of the iteration's KKT solves: autotuned for their shape
    # on whole-body-shaped data of that shape
    host = synth.gen_batch(synth.gen_c3, batch, np.float32)
    dev = {k: torch.from_numpy(v).to("cuda:0") for k, v in host.items()}
    mapping = L.autotune(*[dev[k] for k in L.FIELDS], refine=1, reps=2)
    del dev, host
    log(f"[bench] sqp: solve mapping {mapping}")
    X, U, Lm = start()
    L.sqp_solve(md, X, U, Lm, iters=1)
    torch.cuda.synchronize()
    X, U, Lm = start()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    st, al = L.sqp_solve(md, X, U, Lm, iters=iters)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    alphas = al.cpu().numpy()
    res = {"workload": f"bilinear model, n=36 m=12 N=100, 24 constraints, batch {batch}, FP32",
           "iterations": iters, "ms_per_iteration": ms, "instance_iterations_per_s": batch / ms * 1e3,
           "solve_mapping": mapping,
           "mean_step": float(alphas.mean()), "full_steps_last_iteration": int((alphas[-1] == 1.0).sum()),
           "line_search_rejections": int((st.cpu().numpy() & 32 != 0).sum())}
    log(f"[bench] sqp: {ms:.2f} ms per iteration of {batch} instances")
    return res


def serving_leg(L, n_clients: int, warm_requests: int, sat_requests: int, requests: int, loads=(0.5, 0.7, 0.9),
                graphs: bool = True):
    """Serving mix through the continuous-batching loop: a saturated run
    (every request present at t = 0) gives the capacity; then Poisson
    arrivals at each fraction of it in `loads` give the latency
    distribution (overall and per request shape)."""
    import torch
    import synth
    from paper_2506_07823_amd.serve import GpuBackend, Request, Server, latency_report
    log(f"[bench] serving: generating {n_clients} clients")
    clients = synth.gen_c5_clients(n_clients)
    # each client writes its QP matrices into pinned host memory once; every
    # request ships them (and its own x0) to the device
    pinned = [{k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).pin_memory()
               for k, v in model.items() if k != "x0"} for model, _ in clients]
    total = warm_requests + sat_requests + requests * len(loads) + 1
    # one page-locked block per client holds all its initial states (a
    # request takes a row view): no page-locked allocation per request
    walks = [torch.from_numpy(synth.x0_walk(model, seed, total).astype(np.float32)).pin_memory()
             for model, seed in clients]
    used = [0] * len(clients)
    rng = np.random.default_rng([5, 4])

    def make(count, rate, rid0):
        reqs, t = [], 0.0
        for j in range(count):
            c = int(rng.integers(0, len(clients)))
            if rate:
                t += rng.exponential(1.0 / rate)
            data = dict(pinned[c])
            data["x0"] = walks[c][used[c]]
            used[c] += 1
            reqs.append(Request(rid=rid0 + j, client=c, data=data, arrival=t))
        return reqs

    free, _ = torch.cuda.mem_get_info()
    budget = int(0.5 * free)
    be = GpuBackend(nstreams=4, refine=1, graphs=graphs)

    def phase(count, rate, rid0):
        srv = Server(be, budget, max_batch=64, warm=True)
        done = srv.run(make(count, rate, rid0))
        torch.cuda.synchronize()
        return done, srv

    log(f"[bench] serving: warmup ({warm_requests} requests)")
    phase(warm_requests, None, 0)
    log(f"[bench] serving: saturated run ({sat_requests} requests)")
    done, _ = phase(sat_requests, None, warm_requests)
    cap = latency_report(done)["solves_per_s"]
    out = {"capacity_solves_per_s": cap, "clients": n_clients, "budget_bytes": budget, "graph_replay": graphs,
           "latency": "arrival to device completion, host->device copies included", "loads": {}}
    rid = warm_requests + sat_requests
    for load in loads:
        rate = load * cap
        log(f"[bench] serving: capacity {cap:.0f} solves/s; {requests} Poisson arrivals at {rate:.0f}/s ({load:.0%})")
        done, srv = phase(requests, rate, rid)
        rid += requests
        rep = latency_report(done)
        out["loads"][f"{int(round(100 * load))}pct"] = {
            "offered_per_s": rate, **rep,
            "max_rel_kkt_residual": max(float(r.result["resid"]) for r in done),
            "instances_with_status": sum(int(r.result["status"] != 0) for r in done),
            "warm_started": sum(r.warm for r in done), "batches": len(srv.launch_log),
            "mean_batch": float(np.mean([k for _, k in srv.launch_log])), "peak_admitted_bytes": srv.peak_used}
    out["graph_replays"] = be.graph_replays
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-multi-robot", action="store_true", help="skip the n=m=192 multi-robot workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-mix workload")
    ap.add_argument("--no-latency", action="store_true", help="skip the single-solve latency workload")
    ap.add_argument("--no-sweep", action="store_true", help="skip the whole-body batch-size sweep")
    ap.add_argument("--no-resolve", action="store_true", help="skip the cached-factor re-solve leg")
    ap.add_argument("--no-sqp", action="store_true", help="skip the SQP-iteration leg")
    ap.add_argument("--serving-requests", type=int, default=10000, help="requests per offered load")
    ap.add_argument("--replays", type=int, default=LAT_REPLAYS, help="graph replays of the p50/p99 loop")
    ap.add_argument("--no-tune", action="store_true", help="use the default mapping instead of autotuning it")
    ap.add_argument("--split", action="store_true",
                    help="pin the split schedule (wavefront engine) for the whole-body workload instead of autotuning")
    ap.add_argument("--sequential", action="store_true",
                    help="pin the chunked schedule with chunk 1 and sequential vector passes (the mapping the "
                         "autotuner picks for the whole-body batch) instead of autotuning")
    ap.add_argument("--streams", type=int, default=0,
                    help="with --sequential: also pin the batch split over this many streams")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of graph replays")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates the HBM byte "
                         "counters of a profiler against a known size) and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}): instances are independent and would "
              "shard across GPUs by batch, but only the single-GPU path is built", file=sys.stderr)
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

    wb, fams = measure(L, synth.gen_c3, BATCH, a.steps, a.warmup, a.eager, 1, not a.no_plain, "whole-body",
                       tune=not a.no_tune, pin=({"engine": "wavefront", "fused": 0, "split": True} if a.split else
                                                {"engine": "wavefront", "fused": 0, "split": 2, "chunk": 1, "sweep": 1,
                                                 "fwd_seq": True, "streams": a.streams} if a.sequential else None),
                       replays=a.replays)
    result = {
        "metric": METRIC, "value": wb.pop("value"), "unit": "solves/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": wb.pop("ms_per_step"), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "whole-body-shaped LQR-KKT, n=36 m=12 N=100, batch 4096, FP32 scan + one "
                               "FP64-residual refinement sweep (instances above the 1e-6 refinement tolerance), "
                               "FP64 residual of the returned solution",
                   "batch": BATCH, "N": N_STAGES, "n": NX, "m": NU, "method": "scan",
                   "launch": "eager" if a.eager else "hipGraph replay"},
    }
    wb.pop("steps")
    result.update(wb)
    rf = roofline_of(fams, "alu", PEAK_FP32_VECTOR, "TFLOP/s")
    rf["frac_of_nonpacked_fp32"] = rf["achieved"] * 1e12 / PEAK_FP32_VECTOR_NONPACKED
    rf["peak_nonpacked_fp32"] = PEAK_FP32_VECTOR_NONPACKED / 1e12
    rf["src_hash"] = kernel_src_hash()
    if rf["kernel"] == TRAFFIC["kernel"] and rf["src_hash"] == TRAFFIC["src_hash"]:
        rf["traffic"] = TRAFFIC["bytes_per_launch"]
        rf["traffic_note"] = TRAFFIC["note"]
    result["roofline"] = rf
    if not a.no_multi_robot:
        mr, mfams = measure(L, synth.gen_c4, MR_BATCH, max(5, a.steps // 3), 1, a.eager, 1, not a.no_plain,
                            "multi-robot", tune=not a.no_tune, replays=max(20, a.replays // 4))
        mr["config"] = {"workload": "centralized multi-robot LQR-KKT, n=m=192 N=50, batch 64, FP32 scan on "
                                    "matrix cores + FP64 residual, refinement above 1e-5", "batch": MR_BATCH, "N": 50,
                        "n": 192, "m": 192}
        mr["roofline"] = roofline_of(mfams, "mfma", PEAK_FP32_MFMA, "TFLOP/s")
        mr["roofline"]["src_hash"] = kernel_src_hash()
        if not a.no_cpu:
            log("[bench] multi-robot: CPU oracle baseline")
            mr["cpu_baseline"] = cpu_baseline(synth.gen_c4, 16, MR_BATCH, "multi-robot")
        result["multi_robot"] = mr
    if not a.no_latency:
        result["latency"] = latency_leg(L)
    if not a.no_sweep:
        result["batch_sweep"] = batch_sweep_leg(L)
    if not a.no_resolve:
        result["resolve"] = resolve_leg(L)
    if not a.no_sqp:
        result["sqp"] = sqp_leg(L)
    if not a.no_serving:
        result["serving"] = serving_leg(L, 40, max(100, a.serving_requests // 10), max(200, a.serving_requests // 5),
                                        a.serving_requests)
    if not a.no_cpu:
        log("[bench] whole-body: CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(synth.gen_c3, a.cpu_sample, BATCH, "whole-body")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
