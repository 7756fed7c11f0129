"""The FP64/FP32 oracle against the pins in ``pins.py``, plus planted mistakes.

The planted-mistake tests rebuild the oracle's C source with one plausible
error (a swapped neighbour, a dropped term, a wrong sign, a Gauss-Seidel
in-place update) into a temporary library, and require that at least one pin
rejects each mutant.  The mistakes live only in that temporary copy.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import pins
from paper_2306_03336_amd import inputs


@pytest.fixture(scope="module")
def run64(oracle_mod):
    return lambda u, coeffs, T: oracle_mod.j2d5pt_f64(np.ascontiguousarray(u, dtype=np.float64), coeffs, T)


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle_pin(run64, check):
    check(run64)


def test_thread_count_invariant(oracle_mod):
    coeffs = inputs.dirichlet_weights(9)
    u = inputs.uniform_grid(57, 43, 10, halo=0.3)
    ref = oracle_mod.j2d5pt_f64(u, coeffs, 25, nthreads=1)
    for nt in (2, 3, 8):
        assert np.array_equal(oracle_mod.j2d5pt_f64(u, coeffs, 25, nthreads=nt), ref)


def test_halo_and_padding_untouched(oracle_mod):
    u = inputs.uniform_grid(9, 6, 11, halo=0.7, pitch=13)
    u[:, 8:] = -5.0  # pitch padding
    got = oracle_mod.j2d5pt_f64(u, inputs.EQUAL_WEIGHTS, 7, cols=6)
    assert np.array_equal(got[0], u[0]) and np.array_equal(got[-1], u[-1])
    assert np.array_equal(got[:, 0], u[:, 0]) and np.array_equal(got[:, 7:], u[:, 7:])


def test_T0_is_identity(oracle_mod):
    u = inputs.uniform_grid(5, 5, 1)
    assert np.array_equal(oracle_mod.j2d5pt_f64(u, inputs.EQUAL_WEIGHTS, 0), u)


def test_invalid_args_rejected(oracle_mod):
    u = inputs.uniform_grid(4, 4, 1)
    with pytest.raises(ValueError):
        oracle_mod.j2d5pt_f64(u, inputs.EQUAL_WEIGHTS, -1)


def test_nan_inf_propagate(oracle_mod):
    u = inputs.uniform_grid(9, 9, 2)
    u[5, 5] = np.nan
    u[2, 2] = np.inf
    got = oracle_mod.j2d5pt_f64(u, inputs.EQUAL_WEIGHTS, 2)
    assert np.isnan(got[5, 5]) and np.isnan(got[4, 4]) and np.isnan(got[3, 5])
    assert np.isinf(got[1, 2]) and not np.isnan(got[1, 2])
    assert np.isfinite(got[8, 1])


def test_f32_exact_rational(oracle_mod):
    """Dyadic weights and 8-bit integers stay exact in FP32 for T <= 5 (8 + 3T <= 24 bits)."""
    rng = np.random.default_rng(21)
    for rows, cols in [(4, 6), (7, 3)]:
        u = rng.integers(0, 256, size=(rows + 2, cols + 2)).astype(np.float32)
        coeffs = (0.5, 0.125, 0.125, 0.125, 0.125)
        got = oracle_mod.j2d5pt_f32(u, coeffs, 5)
        want = pins._exact_steps(u.astype(np.float64).tolist(), coeffs, 5)
        assert np.array_equal(got.astype(np.float64), np.array([[float(x) for x in r] for r in want]))


def test_f32_within_float_bound_of_f64(oracle_mod):
    coeffs = inputs.dirichlet_weights(12)
    u = inputs.uniform_grid(40, 33, 13)
    T = 100
    ref = oracle_mod.j2d5pt_f64(u.astype(np.float32).astype(np.float64),
                                np.array(coeffs, dtype=np.float32).astype(np.float64), T)
    got = oracle_mod.j2d5pt_f32(u.astype(np.float32), coeffs, T)
    err = oracle_mod.rel_max_err(got, ref)
    assert err < 6 * T * np.finfo(np.float32).eps
    assert err > 0  # really computed in single precision


# ----------------------------------------------------------------------------- planted mistakes

_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "j2d5pt_oracle.c")

MUTANTS = {
    "swap_n_s": [("acc = acc + ws * up[j];", "acc = acc + ws * dn[j];"),
                 ("acc = acc + wn * dn[j];", "acc = acc + wn * up[j];")],
    "swap_e_w": [("double acc = ww * mid[j - 1];", "double acc = ww * mid[j + 1];"),
                 ("acc = acc + we * mid[j + 1];", "acc = acc + we * mid[j - 1];")],
    "drop_center": [("acc = acc + wc * mid[j];", "")],
    "drop_north": [("acc = acc + wn * dn[j];", "")],
    "minus_west": [("double acc = ww * mid[j - 1];", "double acc = -ww * mid[j - 1];")],
    "weight_mixup": [("const double wc = coeffs[0], wn = coeffs[1], ws = coeffs[2];",
                      "const double wc = coeffs[0], wn = coeffs[2], ws = coeffs[1];")],
    "gauss_seidel": [("double* out = v;", "double* out = u;")],
    "row_off_by_one": [("const double* dn = in + (i + 1) * pitch; /* row i+1: N */",
                        "const double* dn = in + (i + 2) * pitch; /* row i+1: N */")],
    "extra_step": [("for (int64_t t = 0; t < T; ++t) {", "for (int64_t t = 0; t <= T; ++t) {")],
}


def _build_mutant(name, tmp_path):
    src = open(_SRC).read()
    f64_part, rest = src.split("int oracle_j2d5pt_f32", 1)
    for old, new in MUTANTS[name]:
        assert old in f64_part, (name, old)
        f64_part = f64_part.replace(old, new, 1)
    path = tmp_path / f"mut_{name}.c"
    path.write_text(f64_part + "int oracle_j2d5pt_f32" + rest)
    lib = tmp_path / f"libmut_{name}.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-std=c11", str(path), "-o", str(lib)])
    so = ctypes.CDLL(str(lib))
    fn = so.oracle_j2d5pt_f64
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                   ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int]

    def run(u, coeffs, T):
        out = np.ascontiguousarray(u, dtype=np.float64).copy()
        c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
        rc = fn(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.shape[0] - 2, out.shape[1] - 2,
                out.shape[1], c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(T), 1)
        assert rc == 0
        return out
    return run


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_planted_mistake(name, tmp_path):
    run = _build_mutant(name, tmp_path)
    caught = []
    for check in pins.ALL_CHECKS:
        try:
            check(run)
        except AssertionError:
            caught.append(check.__name__)
    assert caught, f"no pin rejects mutant {name}"


# ----------------------------------------------------------------------------- the error measure itself

def test_rel_max_err_known_values(oracle_mod):
    """The relative max-norm over the interior, max|g - o| / max|o|, on hand-built arrays whose answer
    is known: the largest |o| is a negative cell, the largest difference is negative, and the halo
    and the pitch padding hold differences far larger than the interior's that must be ignored."""
    rows, cols, pitch = 3, 4, 8
    o = np.zeros((rows + 2, pitch))
    o[1:rows + 1, 1:cols + 1] = [[0.5, -4.0, 1.0, 2.0],
                                 [1.5, 0.25, -1.0, 3.0],
                                 [0.0, 2.5, 1.25, -0.5]]
    g = o.copy()
    g[2, 3] -= 0.5            # the largest difference, negative: |d| = 0.5
    g[3, 4] += 0.25           # a smaller one
    g[0, :] = 1e6             # halo rows and columns: ignored
    g[:, 0] = -1e6
    g[:, cols + 1] = 1e6
    g[rows + 1, :] = -1e6
    g[:, cols + 2:] = 7e5     # pitch padding: ignored
    # max |o| over the interior is 4.0 (a negative cell); 0.5 / 4.0 = 0.125 exactly.
    assert oracle_mod.rel_max_err(g, o, rows, cols) == 0.125
    # The normalisation is by the reference, not by the result: scaling g's interior changes
    # the numerator only.
    g2 = o.copy()
    g2[1:rows + 1, 1:cols + 1] *= 3.0   # |d| = 2 * 4.0 = 8.0 at the -4.0 cell
    assert oracle_mod.rel_max_err(g2, o, rows, cols) == 2.0
    # Symmetric in the sign of the difference, zero for identical interiors.
    assert oracle_mod.rel_max_err(o, g, rows, cols) == 0.125
    assert oracle_mod.rel_max_err(o.copy(), o, rows, cols) == 0.0
    # A reference whose interior is all zero: the absolute max difference.
    z = np.zeros((rows + 2, cols + 2))
    gz = z.copy()
    gz[2, 2] = -3e-7
    assert oracle_mod.rel_max_err(gz, z) == 3e-7
    # rows/cols default to the reference's storage without padding.
    sq = np.arange(36, dtype=np.float64).reshape(6, 6)   # interior [1:5, 1:5], max |o| = 28
    sq2 = sq.copy()
    sq2[4, 1] += 7.0
    assert oracle_mod.rel_max_err(sq2, sq) == 0.25
