"""Pin strength: plausible mistakes planted in a copy of the oracle are caught.

Each mutant rewrites one spot of ``oracle/lqr_oracle.c`` in a temporary copy
(a dropped term, a flipped sign, a transposed operand, a wrong index, the
misprints of the paper's combine and forward-scan rules), builds it with gcc,
swaps it in, and runs the pin battery of ``test_oracle_pins``.  At least one
pin must fail for every mutant.  The real oracle source is never modified.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "lqr_oracle.c")

MUTANTS = {
    # Riccati recursion, eq. (lqr)
    "G_drops_R": ("G[i] += Rk[i];", "G[i] += 0.0 * Rk[i];"),
    "H_cross_transposed": ("H[i * n + j] += Mk[j * m + i];", "H[i * n + j] += Mk[i * n + j];"),
    "K_sign": ("Kk[i] = -H[i];", "Kk[i] = H[i];"),
    "v_drops_Pc": ("for (int i = 0; i < n; ++i) v[i] += pn[i];", "for (int i = 0; i < n; ++i) v[i] = pn[i];"),
    "p_drops_Kh": ("pk[i] += q[(size_t)k * n + i] + w[i];", "pk[i] += q[(size_t)k * n + i];"),
    "P_A_not_transposed": ("mm(n, n, n, Ak, 1, PA, 0, Pk);", "mm(n, n, n, Ak, 0, PA, 0, Pk);"),
    "rollout_drops_c": ("xn[i] += w[i] + c[(size_t)k * n + i];", "xn[i] += w[i];"),
    "costate_drops_p": ("lam[(size_t)k * n + i] += p[(size_t)k * n + i];", "lam[(size_t)k * n + i] += 0.0;"),
    # dense kernels
    "chol_multiplies": ("S[i * n + j] = s / d;", "S[i * n + j] = s * d;"),
    "cholsolve_backsub_untransposed": ("s -= L[k * n + i] * Y[k * nrhs + c];", "s -= L[i * n + k] * Y[k * nrhs + c];"),
    "lu_forgets_rhs_swap": ("{ double t = Y[j*nrhs+k]; Y[j*nrhs+k] = Y[piv*nrhs+k]; Y[piv*nrhs+k] = t; }", "{ }"),
    # element, eq. (initialization)
    "element_A_sign": ("At[i * n + j] = A[i * n + j] - bs;", "At[i * n + j] = A[i * n + j] + bs;"),
    "element_C_uses_S": ("bb += B[i * m + l] * Y[l * w + n + j];", "bb += M[i * m + l] * Y[l * w + n + j];"),
    "element_p_sign": ("pt[i] = q[i] - sr;", "pt[i] = q[i] + sr;"),
    "element_b_drops": ("bt[i] = c[i] - br;", "bt[i] = c[i];"),
    # combine, eq. (combination_rule)
    "combine_E_transposed": ("mm(n, n, n, C1, 0, P2, 0, E);", "mm(n, n, n, P2, 0, C1, 0, E);"),
    "combine_b_sign": ("Y[i * w + 2 * n] = b1[i] - t[i];", "Y[i * w + 2 * n] = b1[i] + t[i];"),
    "combine_C_A2_untransposed": ("mm(n, n, n, T, 0, A2, 1, C);", "mm(n, n, n, T, 0, A2, 0, C);"),
    "combine_p_printed_sign": ("Z[i * w2 + n] = p2[i] + t[i];", "Z[i * w2 + n] = p2[i] - t[i];"),
    "combine_P_A1_untransposed": ("for (int l = 0; l < n; ++l) s += A1[l * n + i] * Z[l * w2 + j];",
                                  "for (int l = 0; l < n; ++l) s += A1[i * n + l] * Z[l * w2 + j];"),
    "combine_drops_P1": ("P[i * n + j] = s + P1[i * n + j];", "P[i * n + j] = s;"),
    # forward trajectory composition: the printed factor order
    "affine_printed_order": ("mm(n, n, n, M2, 0, M1, 0, M);", "mm(n, n, n, M1, 0, M2, 0, M);"),
    # KKT residual
    "residual_drops_Alam": ("for (int j = 0; j < n; ++j) s += A[k * nn + (size_t)j * n + i] * lam[(size_t)(k + 1) * n + j];",
                            "for (int j = 0; j < n; ++j) s += 0.0 * lam[(size_t)(k + 1) * n + j];"),
}


def battery(lib_module):
    """Run the pin tests with whatever library the oracle module now calls;
    returns the names of the pins that failed."""
    failed = []
    checks = [
        ("golden", lambda: [pins.test_hand_derived_scalar_cases(lib_module, c) for c in pins.load_golden()]),
        ("dense_16_4_2", lambda: pins.test_dense_kkt_matches(lib_module, 16, 4, 2)),
        ("dense_6_6_4", lambda: pins.test_dense_kkt_matches(lib_module, 6, 6, 4)),
        ("residual_operator", lambda: pins.test_residual_function_is_the_kkt_operator(lib_module)),
        ("element_cvf", lambda: pins.test_element_is_one_stage_cvf(lib_module, 4, 2)),
        ("combine_cvf", lambda: pins.test_combine_is_segment_cvf(lib_module, 3, 4, 2)),
        ("combine_cvf_square", lambda: pins.test_combine_is_segment_cvf(lib_module, 2, 3, 3)),
        ("suffix_fold", lambda: pins.test_suffix_fold_is_value_function(lib_module, "rand")),
        ("affine_scan", lambda: pins.test_affine_scan_is_rollout(lib_module)),
    ]
    for name, fn in checks:
        try:
            with np.errstate(all="ignore"):
                fn()
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            failed.append(name)
    return failed


@pytest.fixture(scope="module")
def mutant_dir():
    with tempfile.TemporaryDirectory() as d:
        yield d


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(oracle_lib, mutant_dir, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    mutated = src.replace(old, new, 1)
    cpath = os.path.join(mutant_dir, f"{name}.c")
    sopath = os.path.join(mutant_dir, f"lib{name}.so")
    with open(cpath, "w") as f:
        f.write(mutated)
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-pthread", "-o", sopath, cpath, "-lm"])
    prev = oracle.use_library(oracle.load_library(sopath))
    try:
        failed = battery(oracle)
    finally:
        oracle.use_library(prev)
    assert failed, f"no pin caught mutant {name}"


def test_unmutated_battery_passes(oracle_lib):
    assert battery(oracle) == []
