"""The j3d7pt (3-D seven-point) FP64/FP32 oracle against the pins in ``pins3d.py``, plus planted mistakes.

The planted-mistake tests rebuild the 3-D oracle's C source with one plausible error (two weights swapped, a
term dropped, a wrong sign, a plane or row off by one, an in-place update, an extra step) into a temporary
library and require that at least one pin rejects each mutant.  The mistakes live only in that temporary copy.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import pins3d
from paper_2306_03336_amd import inputs


@pytest.fixture(scope="module")
def run64(oracle_mod):
    return lambda u, coeffs, T: oracle_mod.j3d7pt_f64(np.ascontiguousarray(u, dtype=np.float64), coeffs, T)


@pytest.mark.parametrize("check", pins3d.ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle3d_pin(run64, check):
    check(run64)


def test_thread_count_invariant(oracle_mod):
    coeffs = inputs.weights7(9)
    u = inputs.uniform_grid3(13, 17, 19, 10, halo=0.3)
    ref = oracle_mod.j3d7pt_f64(u, coeffs, 9, nthreads=1)
    for nt in (2, 3, 8):
        assert np.array_equal(oracle_mod.j3d7pt_f64(u, coeffs, 9, nthreads=nt), ref)


def test_halo_and_padding_untouched(oracle_mod):
    u = inputs.uniform_grid3(4, 5, 6, 11, halo=0.7, pitch=11)
    u[:, :, 8:] = -5.0  # pitch padding
    got = oracle_mod.j3d7pt_f64(u, inputs.weights7(1), 5, cols=6)
    assert np.array_equal(got[0], u[0]) and np.array_equal(got[-1], u[-1])
    assert np.array_equal(got[:, 0], u[:, 0]) and np.array_equal(got[:, -1], u[:, -1])
    assert np.array_equal(got[:, :, 0], u[:, :, 0]) and np.array_equal(got[:, :, 7:], u[:, :, 7:])


def test_T0_identity_and_bad_args(oracle_mod):
    u = inputs.uniform_grid3(3, 3, 3, 1)
    assert np.array_equal(oracle_mod.j3d7pt_f64(u, inputs.weights7(1), 0), u)
    with pytest.raises(ValueError):
        oracle_mod.j3d7pt_f64(u, inputs.weights7(1), -1)
    with pytest.raises(ValueError):
        oracle_mod.j3d7pt_f64(u, inputs.EQUAL_WEIGHTS, 1)  # five weights for a seven-point stencil


def test_f32_exact_rational(oracle_mod):
    """Weights with at most 3 fractional bits and 8-bit integers stay exact in FP32 for T <= 5 (8 + 3T <= 24)."""
    rng = np.random.default_rng(37)
    coeffs = (0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125)
    u = rng.integers(0, 256, size=(5, 6, 7)).astype(np.float64)
    want = pins3d._exact_steps(u.tolist(), coeffs, 5)
    got = oracle_mod.j3d7pt_f32(u.astype(np.float32), coeffs, 5)
    for z in range(5):
        for i in range(6):
            for j in range(7):
                assert float(got[z, i, j]) == float(want[z][i][j]), (z, i, j)


def test_f32_within_float_bound_of_f64(oracle_mod):
    """On non-negative weights summing to 1: |f32 - f64| <= (2 * 7 T + 1) u max|u0|, u = 2^-24."""
    coeffs = inputs.weights7(11)
    u = inputs.uniform_grid3(12, 14, 13, 12, halo=0.5)
    T = 40
    ref = oracle_mod.j3d7pt_f64(u, coeffs, T)
    got = oracle_mod.j3d7pt_f32(u.astype(np.float32), coeffs, T).astype(np.float64)
    err = np.max(np.abs(got - ref))
    assert 0 < err <= (2 * 7 * T + 1) * 2.0 ** -24 * np.max(np.abs(u))


# ----------------------------------------------------------------------------- planted mistakes

_SRC = os.path.join(os.path.dirname(__file__), "..", "oracle", "j3d7pt_oracle.c")

MUTANTS = {
    "swap_t_b": [("acc = acc + wb * bel[j];", "acc = acc + wt * bel[j];"),
                 ("acc = acc + wt * abv[j];", "acc = acc + wb * abv[j];")],
    "swap_n_s": [("acc = acc + ws * up[j];", "acc = acc + wn * up[j];"),
                 ("acc = acc + wn * dn[j];", "acc = acc + ws * dn[j];")],
    "drop_top": [("acc = acc + wt * abv[j];", "(void)abv;")],
    "drop_bottom": [("acc = acc + wb * bel[j];", "(void)bel;")],
    "minus_west": [("double acc = ww * mid[j - 1];", "double acc = -ww * mid[j - 1];")],
    "plane_above_is_same": [("const double* abv = in + (z + 1) * plane_pitch + i * pitch; /* plane z+1: T */",
                             "const double* abv = in + z * plane_pitch + i * pitch; /* plane z+1: T */")],
    "below_reads_row_off": [("const double* bel = in + (z - 1) * plane_pitch + i * pitch; /* plane z-1: B */",
                             "const double* bel = in + (z - 1) * plane_pitch + (i - 1) * pitch; /* plane z-1: B */")],
    "weight_mixup": [("const double wt = coeffs[5], wb = coeffs[6];", "const double wt = coeffs[6], wb = coeffs[5];")],
    "gauss_seidel": [("double* out = v;", "double* out = u;")],
    "extra_step": [("for (int64_t t = 0; t < T; ++t) {", "for (int64_t t = 0; t <= T; ++t) {")],
}


def _build_mutant(name, tmp_path):
    src = open(_SRC).read()
    f64_part, rest = src.split("int oracle_j3d7pt_f32", 1)
    for old, new in MUTANTS[name]:
        assert old in f64_part, (name, old)
        f64_part = f64_part.replace(old, new, 1)
    path = tmp_path / f"mut3_{name}.c"
    path.write_text(f64_part + "int oracle_j3d7pt_f32" + rest)
    lib = tmp_path / f"libmut3_{name}.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-std=c11", str(path), "-o", str(lib)])
    so = ctypes.CDLL(str(lib))
    fn = so.oracle_j3d7pt_f64
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                   ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int]

    def run(u, coeffs, T):
        out = np.ascontiguousarray(u, dtype=np.float64).copy()
        c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
        assert c.size == 7
        d, r, p = out.shape
        rc = fn(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d - 2, r - 2, p - 2, p, r * p,
                c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(T), 1)
        assert rc == 0
        return out
    return run


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins3d_reject_planted_mistake(name, tmp_path):
    run = _build_mutant(name, tmp_path)
    caught = []
    for check in pins3d.ALL_CHECKS:
        try:
            check(run)
        except (AssertionError, IndexError, ValueError):
            caught.append(check.__name__)
    assert caught, f"no pin rejects mutant {name}"
