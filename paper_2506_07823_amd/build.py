"""Build liblqr_kkt.so (the HIP/gfx950 C-ABI library) in-tree.

Each (padded-order class, storage type) pair is a separate translation unit, compiled in parallel
with hipcc; the objects are linked against the HIP runtime that PyTorch-ROCm
loads (``torch/lib/libamdhip64.so``), so that a Python process holding both
torch and this library runs a single HIP runtime.

    python paper_2506_07823_amd/build.py [--jobs J] [--no-force]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import importlib.util
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblqr_kkt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
TS_CLASSES = (1, 2, 3, 4, 5, 6, 8, 32)

HIPFLAGS = [
    "-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-c",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def torch_lib_dir() -> str:
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        raise RuntimeError("PyTorch-ROCm is required: its HIP runtime is the one the library links")
    d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so under {d}")
    return d


def _sources():
    deps = [os.path.join(CSRC, f) for f in ("engine.hpp", "bigeng.hpp", "kernels.hpp", "kernels_big.hpp", "runs.hpp", "pack.hpp",
                                            "qpdata.hpp", "sqp.hpp")]
    deps.append(os.path.join(HERE, "..", "include", "lqr_kkt.h"))
    units = [("lqr_kkt", os.path.join(CSRC, "lqr_kkt.hip"), [])]
    # the slowest units first, so the parallel build ends sooner
    for ts in sorted(TS_CLASSES, key=lambda t: -t if t != 32 else 0):
        for sv in ("float", "double"):
            units.append((f"inst_ts{ts}_{sv}", os.path.join(CSRC, "inst.hip"), [f"-DLQR_TS={ts}", f"-DLQR_S={sv}"]))
    return units, deps


def _stale(obj, src, deps):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(p) > t for p in [src] + deps)


def build(force: bool = True, jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units, deps = _sources()
    jobs = jobs or min(16, os.cpu_count() or 4)

    def compile_one(u):
        name, src, extra = u
        obj = os.path.join(BUILD, name + ".o")
        if not force and not _stale(obj, src, deps):
            return obj
        cmd = [HIPCC, *HIPFLAGS, *extra, "-o", obj + ".tmp", src]
        r = subprocess.run(cmd, capture_output=True, text=True)
        errs = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {name}:\n{errs}")
        if verbose and errs.strip():
            print(errs, file=sys.stderr)
        os.replace(obj + ".tmp", obj)
        return obj

    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, units))
    tl = torch_lib_dir()
    tmp = LIB + ".tmp"
    cmd = ["g++", "-shared", "-o", tmp, *objs, f"-L{tl}", "-l:libamdhip64.so",
           f"-Wl,-rpath,{tl}", "-Wl,--no-undefined", "-lstdc++"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--no-force", action="store_true")
    a = ap.parse_args()
    print(build(force=not a.no_force, jobs=a.jobs, verbose=True))


if __name__ == "__main__":
    main()
