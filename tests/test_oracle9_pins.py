"""The j2d9pt (3 x 3 box) FP64/FP32 oracle against the pins in ``pins9.py``, plus planted mistakes.

The planted-mistake tests rebuild the box oracle's C source with one plausible
error (two weights swapped, a corner or a term dropped, a wrong sign, a row or
column off by one, an in-place update, an extra step) into a temporary library
and require that at least one pin rejects each mutant.  The mistakes live only
in that temporary copy.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import pins9
from paper_2306_03336_amd import inputs


@pytest.fixture(scope="module")
def run64(oracle_mod):
    return lambda u, coeffs, T: oracle_mod.j2d9pt_f64(np.ascontiguousarray(u, dtype=np.float64), coeffs, T)


@pytest.mark.parametrize("check", pins9.ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle9_pin(run64, check):
    check(run64)


def test_thread_count_invariant(oracle_mod):
    coeffs = inputs.box_weights(9)
    u = inputs.uniform_grid(57, 43, 10, halo=0.3)
    ref = oracle_mod.j2d9pt_f64(u, coeffs, 25, nthreads=1)
    for nt in (2, 3, 8):
        assert np.array_equal(oracle_mod.j2d9pt_f64(u, coeffs, 25, nthreads=nt), ref)


def test_halo_and_padding_untouched(oracle_mod):
    u = inputs.uniform_grid(9, 6, 11, halo=0.7, pitch=13)
    u[:, 8:] = -5.0  # pitch padding
    got = oracle_mod.j2d9pt_f64(u, inputs.EQUAL_WEIGHTS9, 7, cols=6)
    assert np.array_equal(got[0], u[0]) and np.array_equal(got[-1], u[-1])
    assert np.array_equal(got[:, 0], u[:, 0]) and np.array_equal(got[:, 7:], u[:, 7:])


def test_T0_is_identity_and_bad_args(oracle_mod):
    u = inputs.uniform_grid(5, 5, 1)
    assert np.array_equal(oracle_mod.j2d9pt_f64(u, inputs.EQUAL_WEIGHTS9, 0), u)
    with pytest.raises(ValueError):
        oracle_mod.j2d9pt_f64(u, inputs.EQUAL_WEIGHTS9, -1)
    with pytest.raises(ValueError):
        oracle_mod.j2d9pt_f64(u, inputs.EQUAL_WEIGHTS, 1)  # five weights for a nine-point stencil


def test_reduces_to_j2d5pt_without_corners(oracle_mod):
    """Zero corner weights leave the 5-point stencil; on dyadic data both oracles are exact, so they agree bit
    for bit whatever order each sums in."""
    rng = np.random.default_rng(26)
    u = rng.integers(0, 256, size=(13, 17)).astype(np.float64)
    c, n, s, e, w = 0.25, 0.125, 0.1875, 0.3125, 0.125
    got9 = oracle_mod.j2d9pt_f64(u, (0.0, s, 0.0, w, c, e, 0.0, n, 0.0), 6)
    got5 = oracle_mod.j2d5pt_f64(u, (c, n, s, e, w), 6)
    assert np.array_equal(got9, got5)


def test_f32_exact_rational(oracle_mod):
    """Weights with at most 4 fractional bits and 8-bit integers stay exact in FP32 for T <= 4 (8 + 4T <= 24)."""
    rng = np.random.default_rng(27)
    coeffs = (0.0625, 0.125, 0.0625, 0.125, 0.25, 0.125, 0.0625, 0.125, 0.0625)
    u = rng.integers(0, 256, size=(10, 12)).astype(np.float64)
    want = pins9._exact_steps(u.tolist(), coeffs, 4)
    got = oracle_mod.j2d9pt_f32(u.astype(np.float32), coeffs, 4)
    for i in range(10):
        for j in range(12):
            assert float(got[i, j]) == float(want[i][j]), (i, j)


def test_f32_within_float_bound_of_f64(oracle_mod):
    """FP32 against FP64 on non-negative weights summing to 1: each step adds at most 9 rounding errors of
    relative size u = 2^-24 on top of the propagated ones, so |f32 - f64| <= (2 * 9 T + 1) u max|u0|."""
    coeffs = inputs.box_weights(11)
    u = inputs.uniform_grid(40, 37, 12, halo=0.5)
    T = 50
    ref = oracle_mod.j2d9pt_f64(u, coeffs, T)
    got = oracle_mod.j2d9pt_f32(u.astype(np.float32), coeffs, T).astype(np.float64)
    err = np.max(np.abs(got - ref))
    bound = (2 * 9 * T + 1) * 2.0 ** -24 * np.max(np.abs(u))
    assert err <= bound, (err, bound)
    assert err > 0  # FP32 really rounds


# ----------------------------------------------------------------------------- planted mistakes

_SRC = os.path.join(os.path.dirname(__file__), "..", "oracle", "j2d9pt_oracle.c")

MUTANTS = {
    "swap_ne_nw": [("acc = acc + k[6] * n[j - 1];", "acc = acc + k[8] * n[j - 1];"),
                   ("acc = acc + k[8] * n[j + 1];", "acc = acc + k[6] * n[j + 1];")],
    "swap_se_nw": [("acc = acc + k[2] * s[j + 1];", "acc = acc + k[6] * s[j + 1];"),
                   ("acc = acc + k[6] * n[j - 1];", "acc = acc + k[2] * n[j - 1];")],
    "drop_sw_corner": [("double acc = k[0] * s[j - 1];", "double acc = 0.0;")],
    "drop_ne_corner": [("acc = acc + k[8] * n[j + 1];", "(void)0;")],
    "minus_east": [("acc = acc + k[5] * m[j + 1];", "acc = acc - k[5] * m[j + 1];")],
    "north_row_is_middle": [("const double* n = in + (i + 1) * pitch; /* row i+1 */",
                             "const double* n = in + i * pitch; /* row i+1 */")],
    "corner_column_off": [("acc = acc + k[2] * s[j + 1];", "acc = acc + k[2] * s[j];")],
    "rows_swapped": [("const double* s = in + (i - 1) * pitch; /* row i-1 */",
                      "const double* s = in + (i + 1) * pitch; /* row i-1 */"),
                     ("const double* n = in + (i + 1) * pitch; /* row i+1 */",
                      "const double* n = in + (i - 1) * pitch; /* row i+1 */")],
    "gauss_seidel": [("double* out = v;", "double* out = u;")],
    "extra_step": [("for (int64_t t = 0; t < T; ++t) {", "for (int64_t t = 0; t <= T; ++t) {")],
}


def _build_mutant(name, tmp_path):
    src = open(_SRC).read()
    f64_part, rest = src.split("int oracle_j2d9pt_f32", 1)
    for old, new in MUTANTS[name]:
        assert old in f64_part, (name, old)
        f64_part = f64_part.replace(old, new, 1)
    path = tmp_path / f"mut9_{name}.c"
    path.write_text(f64_part + "int oracle_j2d9pt_f32" + rest)
    lib = tmp_path / f"libmut9_{name}.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-std=c11", str(path), "-o", str(lib)])
    so = ctypes.CDLL(str(lib))
    fn = so.oracle_j2d9pt_f64
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                   ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int]

    def run(u, coeffs, T):
        out = np.ascontiguousarray(u, dtype=np.float64).copy()
        c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
        assert c.size == 9
        rc = fn(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.shape[0] - 2, out.shape[1] - 2,
                out.shape[1], c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(T), 1)
        assert rc == 0
        return out
    return run


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins9_reject_planted_mistake(name, tmp_path):
    run = _build_mutant(name, tmp_path)
    caught = []
    for check in pins9.ALL_CHECKS:
        try:
            check(run)
        except (AssertionError, IndexError, ValueError):
            caught.append(check.__name__)
    assert caught, f"no pin rejects mutant {name}"
