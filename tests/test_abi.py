"""The C-ABI library loads and exports every entry point its header declares
(host-only checks: no compute call needs a GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqr_kkt.h")
LIB = os.path.join(ROOT, "paper_2506_07823_amd", "liblqr_kkt.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lqr_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("lqr_create", "lqr_destroy", "lqr_workspace_size", "lqr_kkt_solve", "lqr_kkt_residual",
              "lqr_opts_default", "lqr_max_dim", "lqr_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python paper_2506_07823_amd/build.py)"
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} not exported"


def test_binding_loads_and_defaults():
    import paper_2506_07823_amd as L
    o = L.default_opts()
    assert o.dtype == L.LQR_F32 and o.method == L.LQR_METHOD_SCAN
    assert o.refine_sweeps == 1 and o.fallback == 1 and o.cond_threshold == 1e6
    o64 = L.lqr_opts()
    L.lqr_opts_default(ctypes.byref(o64), L.LQR_F64)
    assert o64.refine_sweeps == 0
    assert L.lqr_max_dim() >= 36


def test_workspace_size_is_host_only_and_monotone():
    import paper_2506_07823_amd as L
    sz = ctypes.c_size_t()
    o = L.default_opts()
    sizes = []
    for batch in (1, 2, 64):
        assert L.lqr_workspace_size(None, batch, 100, 36, 12, ctypes.byref(o), ctypes.byref(sz)) == 0
        sizes.append(sz.value)
    assert sizes[0] > 0 and sizes[1] > sizes[0] and sizes[2] > sizes[1]
    assert L.lqr_workspace_size(None, 1, 0, 4, 2, ctypes.byref(o), ctypes.byref(sz)) == L.LQR_EINVAL
    assert L.lqr_workspace_size(None, 1, 4, 4000, 2, ctypes.byref(o), ctypes.byref(sz)) == L.LQR_EUNSUPPORTED
    assert b"exceed" in L.lqr_last_error()


def test_solve_rejects_null_handle_without_launching():
    import paper_2506_07823_amd as L
    o = L.default_opts()
    rc = L.lqr_kkt_solve(None, None, 1, 4, 2, 1, *([None] * 9), None, None, None, None, None, 0,
                         ctypes.byref(o))
    assert rc == L.LQR_EINVAL
    assert b"null handle" in L.lqr_last_error()


def _fake_problem(L, N, n, m, base=0x10000):
    """A descriptor with distinct, aligned, never-dereferenced addresses
    (the size and validation calls below are host-only)."""
    p = L.lqr_problem()
    p.N, p.n, p.m = N, n, m
    for i, f in enumerate(("A", "B", "c", "Q", "R", "M", "q", "r", "x0", "x", "u", "lam")):
        setattr(p, f, base + 0x1000 * i)
    return p


def test_ragged_workspace_is_the_largest_group():
    import paper_2506_07823_amd as L
    o = L.default_opts()
    shapes = [(25, 12, 12), (50, 36, 12), (25, 12, 12), (7, 3, 2)]
    table = (L.lqr_problem * len(shapes))(*[_fake_problem(L, *s) for s in shapes])
    sz = ctypes.c_size_t()
    assert L.lqr_ragged_workspace_size(None, len(shapes), table, ctypes.byref(o), ctypes.byref(sz)) == 0
    # the whole-body group alone (one instance) dominates: its batch-of-one
    # workspace plus packed arrays
    one = ctypes.c_size_t()
    assert L.lqr_workspace_size(None, 1, 50, 36, 12, ctypes.byref(o), ctypes.byref(one)) == 0
    assert sz.value > one.value
    # a group of two SRBD-shaped problems needs less than two whole-body ones
    small = (L.lqr_problem * 2)(_fake_problem(L, 25, 12, 12), _fake_problem(L, 25, 12, 12))
    s2 = ctypes.c_size_t()
    assert L.lqr_ragged_workspace_size(None, 2, small, ctypes.byref(o), ctypes.byref(s2)) == 0
    assert s2.value < sz.value


def test_ragged_descriptor_validation():
    import paper_2506_07823_amd as L
    o = L.default_opts()
    sz = ctypes.c_size_t()
    bad = _fake_problem(L, 10, 4, 2)
    bad.B = 0
    t = (L.lqr_problem * 1)(bad)
    assert L.lqr_ragged_workspace_size(None, 1, t, ctypes.byref(o), ctypes.byref(sz)) == L.LQR_EINVAL
    mis = _fake_problem(L, 10, 4, 2)
    mis.A = 0x10002                       # not aligned to 4 bytes
    t = (L.lqr_problem * 1)(mis)
    assert L.lqr_ragged_workspace_size(None, 1, t, ctypes.byref(o), ctypes.byref(sz)) == L.LQR_EINVAL
    t = (L.lqr_problem * 1)(_fake_problem(L, 0, 4, 2))
    assert L.lqr_ragged_workspace_size(None, 1, t, ctypes.byref(o), ctypes.byref(sz)) == L.LQR_EINVAL
    assert L.lqr_ragged_workspace_size(None, 0, t, ctypes.byref(o), ctypes.byref(sz)) == L.LQR_EINVAL


def test_autotune_workspace_covers_both_engines():
    import paper_2506_07823_amd as L
    o = L.default_opts()
    sz, base = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.lqr_autotune_workspace_size(64, 20, 40, 12, ctypes.byref(o), ctypes.byref(sz)) == 0
    assert L.lqr_workspace_size(None, 64, 20, 40, 12, ctypes.byref(o), ctypes.byref(base)) == 0
    assert sz.value > base.value          # room for the matrix-core engine's scratch slots too
