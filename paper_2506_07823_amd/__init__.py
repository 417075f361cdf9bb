"""MI355X (gfx950) LQR-KKT solver: thin Python binding of liblqr_kkt.so.

The solver is the C-ABI library declared in ``include/lqr_kkt.h`` (HIP
kernels in ``csrc/``).  This module only marshals torch tensors (device
memory) and the current torch stream into those calls; every step of the
solve runs in the library's kernels.  There is no CPU fallback: importing
this package raises if the built library is missing.

Functions with the C names (``lqr_create``, ``lqr_workspace_size``,
``lqr_kkt_solve``, ``lqr_kkt_residual``, ...) are exposed as-is; ``solve``
and ``kkt_residual`` wrap them for tensors with a leading batch axis:

    A [B][N][n][n]  B [B][N][n][m]  c [B][N][n]  Q [B][N+1][n][n]  R [B][N][m][m]
    M [B][N][n][m]  q [B][N+1][n]   r [B][N][m]  x0 [B][n]
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch  # loads the HIP runtime the library links against (must come first)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblqr_kkt.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lqr_kkt.h")

LQR_OK, LQR_EINVAL, LQR_ENOMEM, LQR_ENUMERIC, LQR_EDEVICE, LQR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
LQR_F32, LQR_F64 = 0, 1
LQR_METHOD_SCAN, LQR_METHOD_SEQ_RICCATI = 0, 1
ST_NONFINITE, ST_NOT_SPD, ST_P_NOT_SPD, ST_FP64_FALLBACK, ST_BAD_DESC, ST_LS_REJECTED = 1, 2, 4, 8, 16, 32
MODEL_FIELDS = ("A", "B", "c", "P", "V", "xr", "ur", "wx", "wu", "Gx", "Gu", "g0", "mu", "delta", "xhat0")


class lqr_opts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("refine_sweeps", ctypes.c_int32),
        ("fallback", ctypes.c_int32),
        ("cond_threshold", ctypes.c_double),
        ("refine_tol", ctypes.c_double),
        ("resid_out", ctypes.c_void_p),
        ("warm_x", ctypes.c_void_p),
        ("warm_u", ctypes.c_void_p),
        ("warm_lam", ctypes.c_void_p),
        ("sync_status", ctypes.c_int32),
    ]


class lqr_tuning(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_int32), ("fused", ctypes.c_int32), ("big_grid", ctypes.c_int32),
                ("ms", ctypes.c_float), ("split", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("sweep", ctypes.c_int32), ("fwd_seq", ctypes.c_int32), ("streams", ctypes.c_int32)]


class lqr_problem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32), ("reserved", ctypes.c_int32)] + \
        [(f, ctypes.c_void_p) for f in ("A", "B", "c", "Q", "R", "M", "q", "r", "x0", "x", "u", "lam")]


class lqr_bilinear_model(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int64), ("N", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("nc", ctypes.c_int32), ("gamma", ctypes.c_double)] + \
        [(f, ctypes.c_void_p) for f in ("A", "B", "c", "P", "V", "xr", "ur", "wx", "wu", "Gx", "Gu", "g0", "mu",
                                        "delta", "xhat0")]


class LqrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lqr error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2506_07823_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_lib.lqr_opts_default.argtypes = [ctypes.POINTER(lqr_opts), _i32]
_lib.lqr_opts_default.restype = None
_lib.lqr_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
_lib.lqr_create.restype = ctypes.c_int
_lib.lqr_destroy.argtypes = [_vp]
_lib.lqr_destroy.restype = ctypes.c_int
_lib.lqr_workspace_size.argtypes = [_vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(lqr_opts), ctypes.POINTER(_sz)]
_lib.lqr_workspace_size.restype = ctypes.c_int
_lib.lqr_kkt_solve.argtypes = [_vp, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int] + [_vp] * 9 + \
    [_vp, _vp, _vp, _vp, _vp, _sz, ctypes.POINTER(lqr_opts)]
_lib.lqr_kkt_solve.restype = ctypes.c_int
_lib.lqr_kkt_resolve.argtypes = _lib.lqr_kkt_solve.argtypes
_lib.lqr_kkt_resolve.restype = ctypes.c_int
_lib.lqr_kkt_solve_noalloc.argtypes = [_vp, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int] + [_vp] * 9 + \
    [_vp, _vp, _vp, _vp, ctypes.POINTER(lqr_opts)]
_lib.lqr_kkt_solve_noalloc.restype = ctypes.c_int
_lib.lqr_noalloc_workspace_bytes.argtypes = []
_lib.lqr_noalloc_workspace_bytes.restype = _sz
_lib.lqr_kkt_residual.argtypes = [_vp, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32] + \
    [_vp] * 9 + [_vp] * 3 + [_vp, _vp, _sz]
_lib.lqr_kkt_residual.restype = ctypes.c_int
_lib.lqr_set_tuning.argtypes = [_vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32,
                                ctypes.POINTER(lqr_tuning)]
_lib.lqr_set_tuning.restype = ctypes.c_int
_lib.lqr_autotune.argtypes = [_vp, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int] + [_vp] * 9 + \
    [_vp, _vp, _vp, _vp, _vp, _sz, ctypes.POINTER(lqr_opts), ctypes.c_int, ctypes.POINTER(lqr_tuning)]
_lib.lqr_autotune.restype = ctypes.c_int
_lib.lqr_autotune_workspace_size.argtypes = [_i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(lqr_opts), ctypes.POINTER(_sz)]
_lib.lqr_autotune_workspace_size.restype = ctypes.c_int
_lib.lqr_ragged_workspace_size.argtypes = [_vp, _i64, ctypes.POINTER(lqr_problem), ctypes.POINTER(lqr_opts),
                                           ctypes.POINTER(_sz)]
_lib.lqr_ragged_workspace_size.restype = ctypes.c_int
_lib.lqr_kkt_solve_ragged.argtypes = [_vp, _vp, _i64, ctypes.POINTER(lqr_problem), _vp, _vp, _sz,
                                      ctypes.POINTER(lqr_opts)]
_lib.lqr_kkt_solve_ragged.restype = ctypes.c_int
_lib.lqr_ragged_dev_workspace_size.argtypes = [_i64, _i32, _i32, _i32, ctypes.POINTER(lqr_opts), ctypes.POINTER(_sz)]
_lib.lqr_ragged_dev_workspace_size.restype = ctypes.c_int
_lib.lqr_kkt_solve_ragged_dev.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _vp, _sz,
                                          ctypes.POINTER(lqr_opts)]
_lib.lqr_kkt_solve_ragged_dev.restype = ctypes.c_int
_lib.lqr_max_dim.argtypes = []
_lib.lqr_max_dim.restype = ctypes.c_int
_lib.lqr_last_error.argtypes = []
_lib.lqr_last_error.restype = ctypes.c_char_p
_lib.lqr_timing_enable.argtypes = [_vp, ctypes.c_int]
_lib.lqr_timing_enable.restype = ctypes.c_int
_lib.lqr_timing_report.argtypes = [_vp, ctypes.c_char_p, _sz]
_lib.lqr_timing_report.restype = ctypes.c_int
_lib.lqr_kkt_factors.argtypes = [_vp, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32, _vp, _sz,
                                 _vp, _vp, _vp, _vp]
_lib.lqr_kkt_factors.restype = ctypes.c_int
_lib.lqr_qp_build.argtypes = [_vp, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              _i32] + [_vp] * 14
_lib.lqr_qp_build.restype = ctypes.c_int
_lib.lqr_sqp_workspace_size.argtypes = [_vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(lqr_opts), ctypes.POINTER(_sz)]
_lib.lqr_sqp_workspace_size.restype = ctypes.c_int
_lib.lqr_sqp_solve.argtypes = [_vp, _vp, ctypes.POINTER(lqr_bilinear_model), ctypes.c_int, ctypes.c_double, _vp, _vp,
                               _vp, _vp, _vp, _vp, _sz, ctypes.POINTER(lqr_opts)]
_lib.lqr_sqp_solve.restype = ctypes.c_int
_lib.lqr_tuning_save.argtypes = [_vp, ctypes.c_char_p]
_lib.lqr_tuning_save.restype = ctypes.c_int
_lib.lqr_tuning_load.argtypes = [_vp, ctypes.c_char_p]
_lib.lqr_tuning_load.restype = ctypes.c_int

# the C entry points under their own names
lqr_opts_default = _lib.lqr_opts_default
lqr_create = _lib.lqr_create
lqr_destroy = _lib.lqr_destroy
lqr_workspace_size = _lib.lqr_workspace_size
lqr_kkt_solve = _lib.lqr_kkt_solve
lqr_kkt_solve_noalloc = _lib.lqr_kkt_solve_noalloc
lqr_kkt_resolve = _lib.lqr_kkt_resolve
lqr_qp_build = _lib.lqr_qp_build
lqr_sqp_workspace_size = _lib.lqr_sqp_workspace_size
lqr_sqp_solve = _lib.lqr_sqp_solve
lqr_noalloc_workspace_bytes = _lib.lqr_noalloc_workspace_bytes
lqr_kkt_residual = _lib.lqr_kkt_residual
lqr_max_dim = _lib.lqr_max_dim
lqr_last_error = _lib.lqr_last_error
lqr_timing_enable = _lib.lqr_timing_enable
lqr_timing_report = _lib.lqr_timing_report
lqr_set_tuning = _lib.lqr_set_tuning
lqr_autotune = _lib.lqr_autotune
lqr_autotune_workspace_size = _lib.lqr_autotune_workspace_size
lqr_ragged_workspace_size = _lib.lqr_ragged_workspace_size
lqr_kkt_solve_ragged = _lib.lqr_kkt_solve_ragged
lqr_ragged_dev_workspace_size = _lib.lqr_ragged_dev_workspace_size
lqr_kkt_solve_ragged_dev = _lib.lqr_kkt_solve_ragged_dev
lqr_tuning_save = _lib.lqr_tuning_save
lqr_kkt_factors = _lib.lqr_kkt_factors
lqr_tuning_load = _lib.lqr_tuning_load

FIELDS = ("A", "B", "c", "Q", "R", "M", "q", "r", "x0")


def _check(rc):
    if rc != LQR_OK:
        raise LqrError(rc, (_lib.lqr_last_error() or b"").decode())


def default_opts(dtype=torch.float32) -> lqr_opts:
    o = lqr_opts()
    _lib.lqr_opts_default(ctypes.byref(o), LQR_F32 if dtype == torch.float32 else LQR_F64)
    return o


_handles = {}
_hlock = threading.Lock()


def handle(device: int = 0):
    with _hlock:
        h = _handles.get(device)
        if h is None:
            hp = _vp()
            _check(_lib.lqr_create(ctypes.byref(hp), int(device)))
            h = _handles[device] = hp
    return h


def workspace_bytes(batch, N, n, m, opts=None) -> int:
    out = _sz()
    _check(_lib.lqr_workspace_size(handle(torch.cuda.current_device()), batch, N, n, m,
                                   ctypes.byref(opts or default_opts()), ctypes.byref(out)))
    return out.value


def dims_of(A, B):
    """(batch, N, n, m) from A [B][N][n][n] and B [B][N][n][m]."""
    batch, N, n, _ = A.shape
    return batch, N, n, B.shape[-1]


def _validate(tensors, dtype, device):
    for name, t in tensors.items():
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device.type != "cuda" or t.device.index != device:
            raise ValueError(f"{name} must live on cuda:{device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")


def _expect_shapes(d, batch, N, n, m):
    want = {"A": (batch, N, n, n), "B": (batch, N, n, m), "c": (batch, N, n), "Q": (batch, N + 1, n, n),
            "R": (batch, N, m, m), "M": (batch, N, n, m), "q": (batch, N + 1, n), "r": (batch, N, m),
            "x0": (batch, n)}
    for k, s in want.items():
        if tuple(d[k].shape) != s:
            raise ValueError(f"{k} has shape {tuple(d[k].shape)}, expected {s}")


class Workspace:
    """Caller-owned device workspace (grown on demand, reused across calls)."""

    def __init__(self, device=None):
        self.device = torch.cuda.current_device() if device is None else device
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self.buf


_default_ws = {}


def solve(A, B, c, Q, R, M, q, r, x0, *, method: str = "scan", refine: int | None = None,
          fallback: bool = True, cond_threshold: float = 1e6, refine_tol: float | None = None,
          want_resid: bool = False, warm=None, sync_status: bool = False,
          workspace: Workspace | None = None, out=None, stream=None):
    """Batched LQR-KKT solve; returns dict x, u, lam, status (+ resid).

    All tensors are device tensors of one dtype (float32 or float64) with a
    leading batch axis; the call is asynchronous on ``stream`` (default: the
    current torch stream).  ``warm`` = (x, u, lam) starts the scan's
    refinement from that solution (it may be ``out``'s own arrays).
    ``sync_status``: wait for the solve and raise LqrError (LQR_ENUMERIC) if
    an instance failed even after the FP64 fallback."""
    d = dict(A=A, B=B, c=c, Q=Q, R=R, M=M, q=q, r=r, x0=x0)
    dtype = A.dtype
    device = A.device.index
    batch, N, n, m = dims_of(A, B)
    _validate(d, dtype, device)
    _expect_shapes(d, batch, N, n, m)
    o = default_opts(dtype)
    o.method = LQR_METHOD_SCAN if method == "scan" else LQR_METHOD_SEQ_RICCATI
    if refine is not None:
        o.refine_sweeps = int(refine)
    o.fallback = 1 if fallback else 0
    o.cond_threshold = float(cond_threshold)
    if refine_tol is not None:
        o.refine_tol = float(refine_tol)
    o.sync_status = 1 if sync_status else 0
    if out is None:
        out = {
            "x": torch.empty((batch, N + 1, n), dtype=dtype, device=A.device),
            "u": torch.empty((batch, N, m), dtype=dtype, device=A.device),
            "lam": torch.empty((batch, N + 1, n), dtype=dtype, device=A.device),
            "status": torch.empty((batch,), dtype=torch.int32, device=A.device),
        }
    if warm is not None:
        wx, wu, wl = warm
        _validate(dict(warm_x=wx, warm_u=wu, warm_lam=wl), dtype, device)
        for t, s in ((wx, (batch, N + 1, n)), (wu, (batch, N, m)), (wl, (batch, N + 1, n))):
            if tuple(t.shape) != s:
                raise ValueError(f"warm start has shape {tuple(t.shape)}, expected {s}")
        o.warm_x, o.warm_u, o.warm_lam = wx.data_ptr(), wu.data_ptr(), wl.data_ptr()
    if want_resid:
        if "resid" not in out:
            out["resid"] = torch.empty((batch,), dtype=torch.float64, device=A.device)
        o.resid_out = out["resid"].data_ptr()
    h = handle(device)
    nbytes = _sz()
    _check(_lib.lqr_workspace_size(h, batch, N, n, m, ctypes.byref(o), ctypes.byref(nbytes)))
    if workspace is None:
        workspace = _default_ws.setdefault(device, Workspace(device))
    wbuf = workspace.get(nbytes.value)
    s = (stream or torch.cuda.current_stream(device)).cuda_stream
    rc = _lib.lqr_kkt_solve(h, s, batch, N, n, m, *[d[k].data_ptr() for k in FIELDS],
                            out["x"].data_ptr(), out["u"].data_ptr(), out["lam"].data_ptr(),
                            out["status"].data_ptr(), wbuf.data_ptr(), wbuf.numel(), ctypes.byref(o))
    _check(rc)
    return out


def resolve(A, B, c, Q, R, M, q, r, x0, *, out, workspace: Workspace, refine: int | None = None,
            want_resid: bool = False, stream=None):
    """lqr_kkt_resolve: re-solve with the factors the last scan solve of
    these matrices left in `workspace` (only x0, c, q, r changed).  `out` is
    that solve's output dict: its status words enter the call (instances
    the FP64 fallback solved are solved again in FP64), and x, u, lam (and
    resid) are overwritten."""
    d = dict(A=A, B=B, c=c, Q=Q, R=R, M=M, q=q, r=r, x0=x0)
    dtype = A.dtype
    device = A.device.index
    batch, N, n, m = dims_of(A, B)
    _validate(d, dtype, device)
    _expect_shapes(d, batch, N, n, m)
    o = default_opts(dtype)
    if refine is not None:
        o.refine_sweeps = int(refine)
    if want_resid:
        if "resid" not in out:
            out["resid"] = torch.empty((batch,), dtype=torch.float64, device=A.device)
        o.resid_out = out["resid"].data_ptr()
    s = (stream or torch.cuda.current_stream(device)).cuda_stream
    _check(_lib.lqr_kkt_resolve(handle(device), s, batch, N, n, m, *[d[k].data_ptr() for k in FIELDS],
                                out["x"].data_ptr(), out["u"].data_ptr(), out["lam"].data_ptr(),
                                out["status"].data_ptr(), workspace.buf.data_ptr(), workspace.buf.numel(),
                                ctypes.byref(o)))
    return out


def solve_ragged(problems, *, refine: int | None = None, want_resid: bool = False,
                 workspace: Workspace | None = None, stream=None):
    """Ragged batch: a list of problems of mixed (N, n, m), each a dict of
    single-instance device tensors A..x0 (no batch axis), solved in one call.
    Returns (list of dicts x, u, lam; status tensor [count]; residual tensor
    [count] or None), in the order of `problems`."""
    count = len(problems)
    first = problems[0]["A"]
    dtype, device = first.dtype, first.device.index
    table = (lqr_problem * count)()
    outs = []
    for i, pr in enumerate(problems):
        _validate(pr, dtype, device)
        N, n, _ = pr["A"].shape
        m = pr["B"].shape[-1]
        o = {"x": torch.empty((N + 1, n), dtype=dtype, device=first.device),
             "u": torch.empty((N, m), dtype=dtype, device=first.device),
             "lam": torch.empty((N + 1, n), dtype=dtype, device=first.device)}
        _expect_shapes({k: v.unsqueeze(0) for k, v in pr.items()}, 1, N, n, m)
        outs.append(o)
        t = table[i]
        t.N, t.n, t.m = N, n, m
        for f in FIELDS:
            setattr(t, f, pr[f].data_ptr())
        t.x, t.u, t.lam = o["x"].data_ptr(), o["u"].data_ptr(), o["lam"].data_ptr()
    op = default_opts(dtype)
    if refine is not None:
        op.refine_sweeps = int(refine)
    status = torch.empty((count,), dtype=torch.int32, device=first.device)
    resid = None
    if want_resid:
        resid = torch.empty((count,), dtype=torch.float64, device=first.device)
        op.resid_out = resid.data_ptr()
    h = handle(device)
    nbytes = _sz()
    _check(_lib.lqr_ragged_workspace_size(h, count, table, ctypes.byref(op), ctypes.byref(nbytes)))
    if workspace is None:
        workspace = _default_ws.setdefault(device, Workspace(device))
    wbuf = workspace.get(nbytes.value)
    s = (stream or torch.cuda.current_stream(device)).cuda_stream
    _check(_lib.lqr_kkt_solve_ragged(h, s, count, table, status.data_ptr(), wbuf.data_ptr(), wbuf.numel(),
                                     ctypes.byref(op)))
    return outs, status, resid


# lqr_problem_desc of the C ABI (112 bytes)
DESC_DTYPE = np.dtype([("N", "<i4"), ("n", "<i4"), ("m", "<i4"), ("status_idx", "<i4"), ("in_off", "<i8", (9,)),
                       ("out_off", "<i8", (3,))])


def field_sizes(N, n, m):
    """Elements of one instance's input arrays (A, B, c, Q, R, M, q, r, x0) and
    output arrays (x, u, lam)."""
    ins = (N * n * n, N * n * m, N * n, (N + 1) * n * n, N * m * m, N * n * m, (N + 1) * n, N * m, n)
    outs = ((N + 1) * n, N * m, (N + 1) * n)
    return ins, outs


def ragged_layout(shapes):
    """Descriptor table (numpy, DESC_DTYPE) and packed buffer sizes for
    problems of the given (N, n, m) shapes, in order: problem i's arrays
    follow problem i-1's, status_idx = i."""
    descs = np.zeros(len(shapes), dtype=DESC_DTYPE)
    ioff = ooff = 0
    for i, (N, n, m) in enumerate(shapes):
        ins, outs = field_sizes(N, n, m)
        d = descs[i]
        d["N"], d["n"], d["m"], d["status_idx"] = N, n, m, i
        for f, k in enumerate(ins):
            d["in_off"][f] = ioff
            ioff += k
        for f, k in enumerate(outs):
            d["out_off"][f] = ooff
            ooff += k
    return descs, ioff, ooff


def solve_ragged_packed(descs, inbuf, outbuf, status, *, count=None, slots=256, maxN, maxd, refine=None,
                        resid=None, warm=None, workspace: Workspace | None = None, stream=None):
    """lqr_kkt_solve_ragged_dev on device buffers: `descs` a uint8 device
    tensor holding `count` descriptors, `inbuf`/`outbuf` packed device
    buffers of the call's dtype, `status` int32 [count], `resid` optional
    float64 [count], `warm` optional packed buffer triple laid out like
    `outbuf` (x, u, lam: here one buffer given three times is accepted)."""
    dtype = inbuf.dtype
    device = inbuf.device.index
    count = descs.numel() // DESC_DTYPE.itemsize if count is None else count
    o = default_opts(dtype)
    if refine is not None:
        o.refine_sweeps = int(refine)
    if resid is not None:
        o.resid_out = resid.data_ptr()
    if warm is not None:
        o.warm_x, o.warm_u, o.warm_lam = (w.data_ptr() for w in warm)
    nbytes = _sz()
    _check(_lib.lqr_ragged_dev_workspace_size(count, int(slots), int(maxN), int(maxd), ctypes.byref(o),
                                              ctypes.byref(nbytes)))
    if workspace is None:
        workspace = _default_ws.setdefault(device, Workspace(device))
    wbuf = workspace.get(nbytes.value)
    s = (stream or torch.cuda.current_stream(device)).cuda_stream
    _check(_lib.lqr_kkt_solve_ragged_dev(handle(device), s, count, descs.data_ptr(), inbuf.data_ptr(),
                                         outbuf.data_ptr(), status.data_ptr(), int(slots), int(maxN), int(maxd),
                                         wbuf.data_ptr(), wbuf.numel(), ctypes.byref(o)))


def solve_ragged_dev(problems, *, slots=256, refine: int | None = None, want_resid: bool = False,
                     workspace: Workspace | None = None, stream=None):
    """Ragged batch through the persistent device-descriptor form: `problems`
    as for solve_ragged (single-instance device tensors of mixed shapes,
    orders up to 64).  Packs them, builds the descriptor table, solves, and
    returns (list of dicts x, u, lam; status [count]; residual [count] or
    None) in the order of `problems`."""
    count = len(problems)
    first = problems[0]["A"]
    dtype, dev = first.dtype, first.device
    shapes = []
    for pr in problems:
        _validate(pr, dtype, dev.index)
        N, n, _ = pr["A"].shape
        shapes.append((int(N), int(n), int(pr["B"].shape[-1])))
        _expect_shapes({k: v.unsqueeze(0) for k, v in pr.items()}, 1, *shapes[-1])
    descs, nin, nout = ragged_layout(shapes)
    inbuf = torch.empty(max(nin, 1), dtype=dtype, device=dev)
    for pr, d in zip(problems, descs):
        for f, name in enumerate(FIELDS):
            t = pr[name].reshape(-1)
            inbuf[int(d["in_off"][f]):int(d["in_off"][f]) + t.numel()].copy_(t)
    outbuf = torch.empty(max(nout, 1), dtype=dtype, device=dev)
    dtab = torch.from_numpy(descs.view(np.uint8).copy()).to(dev)
    status = torch.empty((count,), dtype=torch.int32, device=dev)
    resid = torch.empty((count,), dtype=torch.float64, device=dev) if want_resid else None
    solve_ragged_packed(dtab, inbuf, outbuf, status, count=count, slots=min(int(slots), count),
                        maxN=max(s[0] for s in shapes), maxd=max(max(s[1], s[2]) for s in shapes), refine=refine,
                        resid=resid, workspace=workspace, stream=stream)
    outs = []
    for (N, n, m), d in zip(shapes, descs):
        o = {}
        for f, (name, shp) in enumerate((("x", (N + 1, n)), ("u", (N, m)), ("lam", (N + 1, n)))):
            off = int(d["out_off"][f])
            o[name] = outbuf[off:off + shp[0] * shp[1]].view(shp)
        outs.append(o)
    return outs, status, resid


def qp_build(Ex, Eu, e, W, Gx=None, Gu=None, g=None, mu=None, delta=None, *, out=None, stream=None) -> dict:
    """lqr_qp_build: Gauss-Newton + relaxed-barrier QP blocks (Q, M, R, q, r
    in the solve's layout) from the residual and constraint Jacobians."""
    dtype, dev = Ex.dtype, Ex.device
    batch, N1, p, n = Ex.shape
    N, m = N1 - 1, Eu.shape[-1]
    nc = 0 if Gx is None else Gx.shape[-2]
    d = dict(Ex=Ex, Eu=Eu, e=e, W=W)
    if nc:
        d.update(Gx=Gx, Gu=Gu, g=g, mu=mu, delta=delta)
    _validate(d, dtype, dev.index)
    want = {"Ex": (batch, N + 1, p, n), "Eu": (batch, N, p, m), "e": (batch, N + 1, p), "W": (batch, N + 1, p, p)}
    if nc:
        want.update(Gx=(batch, N + 1, nc, n), Gu=(batch, N, nc, m), g=(batch, N + 1, nc), mu=(nc,), delta=(nc,))
    for k, shp in want.items():
        if tuple(d[k].shape) != shp:
            raise ValueError(f"{k} has shape {tuple(d[k].shape)}, expected {shp}")
    if out is None:
        out = {"Q": torch.empty((batch, N + 1, n, n), dtype=dtype, device=dev),
               "M": torch.empty((batch, N, n, m), dtype=dtype, device=dev),
               "R": torch.empty((batch, N, m, m), dtype=dtype, device=dev),
               "q": torch.empty((batch, N + 1, n), dtype=dtype, device=dev),
               "r": torch.empty((batch, N, m), dtype=dtype, device=dev)}
    ptr = lambda k: d[k].data_ptr() if k in d else None  # noqa: E731
    s = (stream or torch.cuda.current_stream(dev.index)).cuda_stream
    _check(_lib.lqr_qp_build(handle(dev.index), s, batch, N, n, m, p, nc, LQR_F32 if dtype == torch.float32 else LQR_F64,
                             ptr("Ex"), ptr("Eu"), ptr("e"), ptr("W"), ptr("Gx"), ptr("Gu"), ptr("g"), ptr("mu"),
                             ptr("delta"), *[out[k].data_ptr() for k in ("Q", "M", "R", "q", "r")]))
    return out


def sqp_solve(model: dict, x, u, lam, *, iters: int = 1, theta_max: float = 1e-2, refine: int | None = None,
              want_alpha: bool = True, workspace: Workspace | None = None, stream=None):
    """lqr_sqp_solve: `iters` SQP iterations (linearize, QP blocks, scan solve,
    parallel filter line search, update) of the bilinear model `model` (device
    tensors named as in MODEL_FIELDS plus the float `gamma`) from the iterate
    (x, u, lam), updated in place.  Returns (status [batch], alphas
    [iters][batch] or None)."""
    A = model["A"]
    dtype, dev = A.dtype, A.device
    batch, n, _ = A.shape
    N, m = u.shape[1], u.shape[2]
    nc = model["Gx"].shape[1] if "Gx" in model and model["Gx"] is not None else 0
    _validate({k: model[k] for k in MODEL_FIELDS if k in model and model[k] is not None}, dtype, dev.index)
    _validate(dict(x=x, u=u, lam=lam), dtype, dev.index)
    md = lqr_bilinear_model()
    md.batch, md.N, md.n, md.m, md.nc, md.gamma = batch, N, n, m, nc, float(model["gamma"])
    for f in MODEL_FIELDS:
        t = model.get(f)
        setattr(md, f, t.data_ptr() if t is not None else None)
    o = default_opts(dtype)
    if refine is not None:
        o.refine_sweeps = int(refine)
    nbytes = _sz()
    _check(_lib.lqr_sqp_workspace_size(handle(dev.index), batch, N, n, m, nc, ctypes.byref(o), ctypes.byref(nbytes)))
    if workspace is None:
        workspace = _default_ws.setdefault(dev.index, Workspace(dev.index))
    wbuf = workspace.get(nbytes.value)
    status = torch.empty((batch,), dtype=torch.int32, device=dev)
    alphas = torch.empty((max(iters, 1), batch), dtype=dtype, device=dev) if want_alpha else None
    s = (stream or torch.cuda.current_stream(dev.index)).cuda_stream
    _check(_lib.lqr_sqp_solve(handle(dev.index), s, ctypes.byref(md), int(iters), float(theta_max), x.data_ptr(),
                              u.data_ptr(), lam.data_ptr(), alphas.data_ptr() if alphas is not None else None,
                              status.data_ptr(), wbuf.data_ptr(), wbuf.numel(), ctypes.byref(o)))
    return status, alphas


def kkt_residual(A, B, c, Q, R, M, q, r, x0, x, u, lam, *, workspace=None, stream=None):
    """FP64 relative KKT residual per instance of a given (x, u, lam)."""
    d = dict(A=A, B=B, c=c, Q=Q, R=R, M=M, q=q, r=r, x0=x0, x=x, u=u, lam=lam)
    dtype = A.dtype
    device = A.device.index
    batch, N, n, m = dims_of(A, B)
    _validate(d, dtype, device)
    rel = torch.empty((batch,), dtype=torch.float64, device=A.device)
    h = handle(device)
    o = default_opts(dtype)
    nbytes = _sz()
    _check(_lib.lqr_workspace_size(h, batch, N, n, m, ctypes.byref(o), ctypes.byref(nbytes)))
    if workspace is None:
        workspace = _default_ws.setdefault(device, Workspace(device))
    wbuf = workspace.get(nbytes.value)
    s = (stream or torch.cuda.current_stream(device)).cuda_stream
    _check(_lib.lqr_kkt_residual(h, s, batch, N, n, m, LQR_F32 if dtype == torch.float32 else LQR_F64,
                                 *[d[k].data_ptr() for k in FIELDS + ("x", "u", "lam")],
                                 rel.data_ptr(), wbuf.data_ptr(), wbuf.numel()))
    return rel


def autotune(A, B, c, Q, R, M, q, r, x0, *, method: str = "scan", refine: int | None = None, reps: int = 3,
             stream=None) -> dict:
    """Time every candidate mapping of this problem shape on these inputs
    and pin the fastest on the device's handle (later solves of the same
    shape use it).  Returns the chosen mapping and its mean solve time."""
    d = dict(A=A, B=B, c=c, Q=Q, R=R, M=M, q=q, r=r, x0=x0)
    dtype = A.dtype
    device = A.device.index
    batch, N, n, m = dims_of(A, B)
    _validate(d, dtype, device)
    _expect_shapes(d, batch, N, n, m)
    o = default_opts(dtype)
    o.method = LQR_METHOD_SCAN if method == "scan" else LQR_METHOD_SEQ_RICCATI
    if refine is not None:
        o.refine_sweeps = int(refine)
    nbytes = _sz()
    _check(_lib.lqr_autotune_workspace_size(batch, N, n, m, ctypes.byref(o), ctypes.byref(nbytes)))
    ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=A.device)
    out = [torch.empty((batch, N + 1, n), dtype=dtype, device=A.device),
           torch.empty((batch, N, m), dtype=dtype, device=A.device),
           torch.empty((batch, N + 1, n), dtype=dtype, device=A.device),
           torch.empty((batch,), dtype=torch.int32, device=A.device)]
    best = lqr_tuning()
    s = (stream or torch.cuda.current_stream(device)).cuda_stream
    _check(_lib.lqr_autotune(handle(device), s, batch, N, n, m, *[d[k].data_ptr() for k in FIELDS],
                             *[t.data_ptr() for t in out], ws.data_ptr(), ws.numel(), ctypes.byref(o), int(reps),
                             ctypes.byref(best)))
    return {"engine": {1: "wavefront", 2: "matrix-core"}[best.engine], "fused": int(best.fused),
            "big_grid": int(best.big_grid), "split": int(best.split), "chunk": int(best.chunk),
            "sweep": int(best.sweep), "fwd_seq": int(best.fwd_seq), "streams": int(best.streams),
            "ms": float(best.ms)}


def set_tuning(batch: int, N: int, n: int, m: int, dtype=torch.float32, *, engine: str | None = None,
               fused: bool | int | None = None, big_grid: int = 0, split: bool | int = False, chunk: int = 0,
               sweep: int = 0, fwd_seq: bool = False, streams: int = 0, device: int = 0, clear: bool = False):
    """Pin (or clear) the mapping of a problem shape on the device's handle.

    fused: None = default; 0 / False = vector-only passes level by level;
    1 / True = one workgroup per instance for them; 2 = the whole solve in
    one launch (wavefront engine).  split: schedule of the reverse scan,
    0 / False = balanced tree, 1 / True = split (tree over the first 2^k
    elements, a sequential sweep over the rest), 2 = chunked (`sweep`
    elements swept sequentially, chunks of `chunk` elements over the rest);
    wavefront engine, fused 0 or 1.  fwd_seq: sequential forward and
    refinement vector passes (no forward-tree products).  streams: 2..4
    splits the batch into that many contiguous parts whose launch sequences
    run on forked streams (0 or 1: one stream)."""
    dt = LQR_F32 if dtype == torch.float32 else LQR_F64
    if clear:
        _check(_lib.lqr_set_tuning(handle(device), batch, N, n, m, dt, None))
        return
    t = lqr_tuning()
    t.engine = {None: 0, "wavefront": 1, "matrix-core": 2}[engine]
    t.fused = -1 if fused is None else int(fused)
    t.big_grid = int(big_grid)
    t.split = int(split)
    t.chunk = int(chunk)
    t.sweep = int(sweep)
    t.fwd_seq = 1 if fwd_seq else 0
    t.streams = int(streams)
    _check(_lib.lqr_set_tuning(handle(device), batch, N, n, m, dt, ctypes.byref(t)))


def save_tuning(path: str, device: int = 0):
    """Write the autotuned mappings (per shape bucket) of the device's handle to `path`."""
    _check(_lib.lqr_tuning_save(handle(device), os.fsencode(path)))


def load_tuning(path: str, device: int = 0) -> int:
    """Load the mappings of this device's architecture from `path`; returns how many."""
    rc = _lib.lqr_tuning_load(handle(device), os.fsencode(path))
    if rc < 0:
        _check(rc)
    return rc


def factors(batch, N, n, m, dtype, workspace: Workspace, stream=None) -> dict:
    """P_k, p_k, K_k, kff_k of the last scan solve of this shape that used
    `workspace` (diagnostics: the records the reverse scan and the policy
    left there)."""
    device = workspace.device
    dev = f"cuda:{device}"
    out = {"P": torch.empty((batch, N + 1, n, n), dtype=dtype, device=dev),
           "p": torch.empty((batch, N + 1, n), dtype=dtype, device=dev),
           "K": torch.empty((batch, N, m, n), dtype=dtype, device=dev),
           "kff": torch.empty((batch, N, m), dtype=dtype, device=dev)}
    s = (stream or torch.cuda.current_stream(device)).cuda_stream
    _check(_lib.lqr_kkt_factors(handle(device), s, batch, N, n, m, LQR_F32 if dtype == torch.float32 else LQR_F64,
                                workspace.buf.data_ptr(), workspace.buf.numel(), out["P"].data_ptr(),
                                out["p"].data_ptr(), out["K"].data_ptr(), out["kff"].data_ptr()))
    return out


def kernel_timing(enable: bool, device: int = 0):
    """Turn per-launch event timing of this device's handle on or off."""
    _check(_lib.lqr_timing_enable(handle(device), 1 if enable else 0))


def kernel_report(device: int = 0) -> dict:
    """Per kernel family: launches, total ms, algorithmic flops (the method's
    per-unit cost model) and bytes, and the flops with the combines counted
    at the minimal cost of the form the kernels execute, of the launches timed since
    the last report (waits for them)."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_lib.lqr_timing_report(handle(device), buf, len(buf)))
    fams = {}
    for line in buf.value.decode().strip().splitlines():
        name, launches, ms, fl, by, flm = line.split()
        fams[name] = dict(launches=int(launches), ms=float(ms), flops=float(fl), bytes=float(by),
                          flops_min=float(flm))
    return fams
