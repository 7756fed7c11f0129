"""CPU oracle for the iterative stencils -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code with it.

``liboracle.so`` holds the plain C loops of ``j2d5pt_oracle.c`` (Listing 1 of
the paper, repeated T times as Section 3.1 and Figure 1 describe) and
``j2d9pt_oracle.c`` (the 3 x 3 box, the next shape of the same method; its
weight order and summation order are that file's stated reading) and
``j3d7pt_oracle.c`` (the 3-D seven-point stencil, likewise).  This module
only loads them and marshals numpy arrays; it holds no stencil arithmetic of
its own.  ``liboracle.so`` is compiled by ``__graft_entry__.build()`` (gcc,
``-O2 -fopenmp -ffp-contract=off``); ``build_if_missing()`` repeats that
command when the library is absent.

Array convention (same as the C file): a 2-D array of shape
(rows + 2, pitch), row-major, interior ``[1:rows+1, 1:cols+1]``, one-cell
Dirichlet halo around it.  j2d5pt coefficients are ordered (c, n, s, e, w);
j2d9pt coefficients (sw, s, se, w, c, e, nw, n, ne), S = row i-1, N = row i+1.
j3d7pt grids are 3-D arrays of shape (depth + 2, rows + 2, pitch) (plane z,
row i, column j), coefficients (c, n, s, e, w, t, b), T = plane z+1, B = z-1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "j2d5pt_oracle.c")
SRC9_PATH = os.path.join(_HERE, "j2d9pt_oracle.c")
SRC3D_PATH = os.path.join(_HERE, "j3d7pt_oracle.c")

# The one compile line for the oracle (also used by __graft_entry__.build()).
GCC_CMD = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-std=c11", SRC_PATH, SRC9_PATH, SRC3D_PATH, "-o", LIB_PATH]

_lib = None


def build_if_missing() -> None:
    if not os.path.exists(LIB_PATH):
        subprocess.check_call(GCC_CMD)


def _load():
    global _lib
    if _lib is None:
        build_if_missing()
        lib = ctypes.CDLL(LIB_PATH)
        for name, ptr_t in (("oracle_j2d5pt_f64", ctypes.c_double),
                            ("oracle_j2d5pt_f32", ctypes.c_float),
                            ("oracle_j2d9pt_f64", ctypes.c_double),
                            ("oracle_j2d9pt_f32", ctypes.c_float)):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.POINTER(ptr_t), ctypes.c_int64, ctypes.c_int64,
                           ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                           ctypes.c_int64, ctypes.c_int]
        for name, ptr_t in (("oracle_j3d7pt_f64", ctypes.c_double), ("oracle_j3d7pt_f32", ctypes.c_float)):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.POINTER(ptr_t), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                           ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                           ctypes.c_int64, ctypes.c_int]
        lib.oracle_default_threads.restype = ctypes.c_int
        lib.oracle_default_threads.argtypes = []
        _lib = lib
    return _lib


def default_threads() -> int:
    return int(_load().oracle_default_threads())


def _run(u: np.ndarray, rows: int, cols: int, coeffs, T: int, nthreads: int,
         dtype, name: str, ctype) -> np.ndarray:
    if u.dtype != dtype or u.ndim != 2:
        raise TypeError(f"expected a 2-D {np.dtype(dtype).name} array")
    if u.shape[0] != rows + 2 or u.shape[1] < cols + 2:
        raise ValueError("array shape does not hold a (rows+2) x (cols+2) grid")
    out = np.ascontiguousarray(u).copy()
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).reshape(9 if "j2d9pt" in name else 5))
    rc = getattr(_load(), name)(out.ctypes.data_as(ctypes.POINTER(ctype)), rows, cols,
                                out.shape[1], c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                int(T), int(nthreads))
    if rc != 0:
        raise ValueError(f"{name} returned {rc}")
    return out


def j2d5pt_f64(u: np.ndarray, coeffs, T: int, nthreads: int = 0, cols: int | None = None) -> np.ndarray:
    """Return u advanced T steps in FP64 (a new array; the halo is copied unchanged)."""
    rows = u.shape[0] - 2
    cols = u.shape[1] - 2 if cols is None else cols
    return _run(u, rows, cols, coeffs, T, nthreads, np.float64, "oracle_j2d5pt_f64", ctypes.c_double)


def j2d5pt_f32(u: np.ndarray, coeffs, T: int, nthreads: int = 0, cols: int | None = None) -> np.ndarray:
    """Return u advanced T steps with every operation in FP32 (coefficients rounded to float)."""
    rows = u.shape[0] - 2
    cols = u.shape[1] - 2 if cols is None else cols
    return _run(u, rows, cols, coeffs, T, nthreads, np.float32, "oracle_j2d5pt_f32", ctypes.c_float)


def j2d9pt_f64(u: np.ndarray, coeffs, T: int, nthreads: int = 0, cols: int | None = None) -> np.ndarray:
    """The 3 x 3 box: u advanced T steps in FP64 (a new array; the halo, corners included, is copied unchanged)."""
    rows = u.shape[0] - 2
    cols = u.shape[1] - 2 if cols is None else cols
    return _run(u, rows, cols, coeffs, T, nthreads, np.float64, "oracle_j2d9pt_f64", ctypes.c_double)


def j2d9pt_f32(u: np.ndarray, coeffs, T: int, nthreads: int = 0, cols: int | None = None) -> np.ndarray:
    """The 3 x 3 box with every operation in FP32 (coefficients rounded to float)."""
    rows = u.shape[0] - 2
    cols = u.shape[1] - 2 if cols is None else cols
    return _run(u, rows, cols, coeffs, T, nthreads, np.float32, "oracle_j2d9pt_f32", ctypes.c_float)


def _run3(u: np.ndarray, coeffs, T: int, nthreads: int, cols, dtype, name: str, ctype) -> np.ndarray:
    if u.dtype != dtype or u.ndim != 3:
        raise TypeError(f"expected a 3-D {np.dtype(dtype).name} array")
    depth, rows = u.shape[0] - 2, u.shape[1] - 2
    cols = u.shape[2] - 2 if cols is None else cols
    out = np.ascontiguousarray(u).copy()
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).reshape(7))
    pitch = out.shape[2]
    rc = getattr(_load(), name)(out.ctypes.data_as(ctypes.POINTER(ctype)), depth, rows, cols, pitch,
                                out.shape[1] * pitch, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                int(T), int(nthreads))
    if rc != 0:
        raise ValueError(f"{name} returned {rc}")
    return out


def j3d7pt_f64(u: np.ndarray, coeffs, T: int, nthreads: int = 0, cols: int | None = None) -> np.ndarray:
    """The 3-D seven-point stencil: u (depth+2, rows+2, pitch) advanced T steps in FP64 (a new array)."""
    return _run3(u, coeffs, T, nthreads, cols, np.float64, "oracle_j3d7pt_f64", ctypes.c_double)


def j3d7pt_f32(u: np.ndarray, coeffs, T: int, nthreads: int = 0, cols: int | None = None) -> np.ndarray:
    """The 3-D seven-point stencil with every operation in FP32 (coefficients rounded to float)."""
    return _run3(u, coeffs, T, nthreads, cols, np.float32, "oracle_j3d7pt_f32", ctypes.c_float)


def rel_max_err(got: np.ndarray, ref: np.ndarray, rows: int | None = None, cols: int | None = None) -> float:
    """Relative max-norm error over the interior: max|g - o| / max|o| (absolute if max|o| == 0)."""
    rows = ref.shape[0] - 2 if rows is None else rows
    cols = ref.shape[1] - 2 if cols is None else cols
    g = np.asarray(got, dtype=np.float64)[1:rows + 1, 1:cols + 1]
    o = np.asarray(ref, dtype=np.float64)[1:rows + 1, 1:cols + 1]
    den = float(np.max(np.abs(o))) if o.size else 0.0
    num = float(np.max(np.abs(g - o))) if o.size else 0.0
    return num / den if den > 0 else num
