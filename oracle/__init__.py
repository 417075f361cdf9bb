"""CPU FP64 oracle for the LQR KKT solve (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU product path never imports it,
links it or calls it, and the two share no code: the only thing they have in
common is the seeded input generator module ``synth``, which holds no
arithmetic of the method.

The arithmetic lives in ``lqr_oracle.c`` (plain C, FP64, naive loops), built
with gcc into ``liblqr_oracle.so`` next to this file.  This module only
marshals numpy arrays into it.  See the C file for the passage of the paper
each function follows:

  riccati          Sec. II-C, eq. (lqr), forward pass, costates
  riccati_batch    the same over independent instances, on host threads
  kkt_residual     Sec. II-B, stationarity of the Lagrangian + constraints
  element          Sec. II-D, eq. (initialization)
  combine          Sec. II-D, eq. (combination_rule) (corrected reading)
  affine_combine   Sec. II-D, composition of conditional optimal trajectories
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lqr_oracle.c")
_LIB = os.path.join(_HERE, "liblqr_oracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O3", "-march=x86-64-v3", "-fPIC", "-shared", "-pthread", "-Wall"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (always when ``force``)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_native(path: str) -> str:
    """Compile the same source for the host it runs on (-march=native) into
    ``path`` (the CPU baseline's timing build; the default build above stays
    portable because the built library travels to other hosts)."""
    flags = [f for f in CFLAGS if not f.startswith("-march=")] + ["-march=native"]
    subprocess.check_call(["gcc", *flags, "-o", path, _SRC, "-lm"])
    return path


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    i, i64 = ctypes.c_int, ctypes.c_int64
    lib.lqro_riccati.argtypes = [i, i, i] + [dp] * 9 + [dp] * 3 + [dp] * 4
    lib.lqro_riccati.restype = i
    lib.lqro_riccati_batch.argtypes = [i64, i, i, i] + [dp] * 9 + [dp] * 3 + [ip, i]
    lib.lqro_riccati_batch.restype = i64
    lib.lqro_kkt_residual.argtypes = [i, i, i] + [dp] * 9 + [dp] * 3 + [dp, dp]
    lib.lqro_kkt_residual.restype = None
    lib.lqro_element.argtypes = [i, i] + [dp] * 8 + [dp] * 5
    lib.lqro_element.restype = i
    lib.lqro_combine.argtypes = [i] + [dp] * 15
    lib.lqro_combine.restype = i
    lib.lqro_affine_combine.argtypes = [i] + [dp] * 6
    lib.lqro_affine_combine.restype = None
    return lib


def load_library(path: str):
    """Bind an oracle shared library at ``path`` (the default one, or a copy
    built from a deliberately mutated source in the pin-strength tests)."""
    return _bind(ctypes.CDLL(path))


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=True)
            _lib = load_library(_LIB)
    return _lib


def use_library(lib):
    """Swap the library the module-level functions call; returns the old one."""
    global _lib
    with _lock:
        old, _lib = _lib, lib
    return old


FIELDS = ("A", "B", "c", "Q", "R", "M", "q", "r", "x0")


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def dims(prob):
    """(N, n, m) of a single-instance problem dict."""
    N, n, m = prob["B"].shape[-3:]
    return N, n, m


def riccati(prob, want_factors: bool = False):
    """Sequential Riccati solve of one instance; returns dict x, u, lam
    (+ P, p, K, kff when ``want_factors``)."""
    lib = _load()
    N, n, m = dims(prob)
    a = {k: _f64(prob[k]) for k in FIELDS}
    x = np.zeros((N + 1, n)); u = np.zeros((N, m)); lam = np.zeros((N + 1, n))
    P = np.zeros((N + 1, n, n)) if want_factors else None
    p = np.zeros((N + 1, n)) if want_factors else None
    K = np.zeros((N, m, n)) if want_factors else None
    kf = np.zeros((N, m)) if want_factors else None
    rc = lib.lqro_riccati(N, n, m, *[_ptr(a[k]) for k in FIELDS], _ptr(x), _ptr(u), _ptr(lam),
                          _ptr(P), _ptr(p), _ptr(K), _ptr(kf))
    if rc != 0:
        raise ValueError(f"oracle riccati failed rc={rc}")
    out = {"x": x, "u": u, "lam": lam}
    if want_factors:
        out.update(P=P, p=p, K=K, kff=kf)
    return out


def riccati_batch(probs, nthreads: int = 1):
    """Batched solve; ``probs`` holds arrays with a leading batch axis.
    Returns (x, u, lam, status)."""
    lib = _load()
    batch = probs["x0"].shape[0]
    N, n, m = probs["B"].shape[1:]
    a = {k: _f64(probs[k]) for k in FIELDS}
    x = np.zeros((batch, N + 1, n)); u = np.zeros((batch, N, m)); lam = np.zeros((batch, N + 1, n))
    st = np.zeros(batch, dtype=np.int32)
    lib.lqro_riccati_batch(batch, N, n, m, *[_ptr(a[k]) for k in FIELDS], _ptr(x), _ptr(u),
                           _ptr(lam), st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           int(nthreads))
    return x, u, lam, st


def kkt_residual(prob, x, u, lam):
    """Stacked KKT residual of one instance and the norms
    (||res||_2, ||(x0, c, q, r)||_2)."""
    lib = _load()
    N, n, m = dims(prob)
    a = {k: _f64(prob[k]) for k in FIELDS}
    x, u, lam = _f64(x), _f64(u), _f64(lam)
    res = np.zeros(n + N * n + (N + 1) * n + N * m)
    norms = np.zeros(2)
    lib.lqro_kkt_residual(N, n, m, *[_ptr(a[k]) for k in FIELDS], _ptr(x), _ptr(u), _ptr(lam),
                          _ptr(res), _ptr(norms))
    return res, float(norms[0]), float(norms[1])


def rel_kkt_residual(prob, x, u, lam) -> float:
    """||r(x, u, lam)||_2 / ||(x0, c, q, r)||_2 of one instance."""
    _, nr, nb = kkt_residual(prob, x, u, lam)
    return nr / nb if nb > 0 else nr


def element(A, B, c, Q, R, M, q, r):
    """One-stage conditional value function (At, bt, Ct, Pt, pt)."""
    lib = _load()
    n, m = B.shape
    ins = [_f64(v) for v in (A, B, c, Q, R, M, q, r)]
    At = np.zeros((n, n)); bt = np.zeros(n); Ct = np.zeros((n, n)); Pt = np.zeros((n, n)); pt = np.zeros(n)
    rc = lib.lqro_element(n, m, *[_ptr(v) for v in ins], _ptr(At), _ptr(bt), _ptr(Ct), _ptr(Pt), _ptr(pt))
    if rc != 0:
        raise ValueError(f"oracle element failed rc={rc}")
    return At, bt, Ct, Pt, pt


def terminal_element(QN, qN):
    n = QN.shape[0]
    return np.zeros((n, n)), np.zeros(n), np.zeros((n, n)), _f64(QN).copy(), _f64(qN).copy()


def combine(e1, e2):
    """e1 (earlier segment) (x) e2 (later segment); elements are tuples
    (A, b, C, P, p)."""
    lib = _load()
    n = e1[0].shape[0]
    a1 = [_f64(v) for v in e1]; a2 = [_f64(v) for v in e2]
    A = np.zeros((n, n)); b = np.zeros(n); C = np.zeros((n, n)); P = np.zeros((n, n)); p = np.zeros(n)
    rc = lib.lqro_combine(n, *[_ptr(v) for v in a1], *[_ptr(v) for v in a2],
                          _ptr(A), _ptr(b), _ptr(C), _ptr(P), _ptr(p))
    if rc != 0:
        raise ValueError(f"oracle combine failed rc={rc}")
    return A, b, C, P, p


def affine_combine(f1, f2):
    """Compose the earlier affine map f1 = (M1, v1) with the later f2."""
    lib = _load()
    n = f1[0].shape[0]
    M1, v1 = _f64(f1[0]), _f64(f1[1]); M2, v2 = _f64(f2[0]), _f64(f2[1])
    M = np.zeros((n, n)); v = np.zeros(n)
    lib.lqro_affine_combine(n, _ptr(M1), _ptr(v1), _ptr(M2), _ptr(v2), _ptr(M), _ptr(v))
    return M, v


def stage(prob, k):
    """Stage-k slices (A, B, c, Q, R, M, q, r) of a single-instance problem."""
    return tuple(prob[f][k] for f in ("A", "B", "c", "Q", "R", "M", "q", "r"))
