"""dtb_run_noalloc (the allocation-free entry point) through the C ABI against dtb_run, the entry point it
is a variant of: the same results bit for bit (the fused chain per cell does not depend on the tiling), and
within 1e-13 of the FP64 oracle; two calls in a row, the second on a smaller grid, then a third on a larger
FP32 grid; the error word stays clear.  Also: its refusals (too large for the fixed area, invalid
arguments) before any launch."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2306_03336_amd import dtb, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _noalloc(g, coeffs, T, err=None):
    lib = dtb.load()
    grid = dtb._grid(g)
    errp = ctypes.c_void_p(err.data_ptr()) if err is not None else None
    rc = lib.dtb_run_noalloc(ctypes.byref(grid), dtb._coeffs(coeffs), int(T), dtb._dtype_of(g), errp,
                             dtb._stream(None))
    return rc


def _case(rows, cols, T, dtype, seed):
    coeffs = inputs.dirichlet_weights(seed)
    u = inputs.uniform_grid(rows, cols, seed + 1, halo=0.25).astype(dtype)
    ga = torch.from_numpy(u).to("cuda")
    gb = ga.clone()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    _say("noalloc", rows, cols, T, np.dtype(dtype).name)
    assert _noalloc(ga, coeffs, T, err) == 0
    dtb.run(gb, coeffs, T)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    a, b = ga.cpu().numpy(), gb.cpu().numpy()
    assert np.array_equal(a, b), (rows, cols, T, float(np.max(np.abs(a.astype(np.float64) - b))))
    ref = oracle.j2d5pt_f64(u.astype(np.float64), np.array(coeffs, dtype=dtype).astype(np.float64), T)
    tol = 1e-13 if dtype == np.float64 else 2 * (6 * T + 1) * 2.0 ** -24
    assert oracle.rel_max_err(a, ref) <= tol


def test_noalloc_matches_dtb_run_two_calls_then_smaller_then_larger():
    _case(900, 1100, 57, np.float64, 11)     # several tiles, ragged edges
    _case(130, 70, 23, np.float64, 12)       # second call: smaller (one tile narrower than the tile)
    _case(1500, 1300, 40, np.float32, 13)    # third: another precision, larger
    _case(1, 1, 5, np.float64, 14)


def test_noalloc_refusals():
    lib = dtb.load()
    c = dtb._coeffs(inputs.EQUAL_WEIGHTS)
    big = torch.zeros((1602, 1602), dtype=torch.float64, device="cuda")   # 1600^2 FP64: over 18 MiB
    g = dtb._grid(big)
    assert lib.dtb_run_noalloc(ctypes.byref(g), c, 3, dtb.F64, None, dtb._stream(None)) == -2
    g = dtb.Grid(0, 5, 5, 7)
    assert lib.dtb_run_noalloc(ctypes.byref(g), c, 3, dtb.F64, None, dtb._stream(None)) == -1
    small = torch.zeros((7, 7), dtype=torch.float64, device="cuda")
    g = dtb._grid(small)
    assert lib.dtb_run_noalloc(ctypes.byref(g), c, 0, dtb.F64, None, dtb._stream(None)) == 0
