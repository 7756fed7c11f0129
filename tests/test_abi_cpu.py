"""libdtb's C ABI without a GPU: it loads, exports what include/*.h declares,
and rejects invalid arguments before making any HIP call."""
import ctypes
import glob
import os
import re

import pytest

from paper_2306_03336_amd import dtb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(dtb_[a-z0-9_]+)\s*\(", text))
    return names


def test_exports_every_declared_symbol():
    lib = dtb.load()
    declared = _declared()
    assert {"dtb_plan", "dtb_run", "dtb_run_batched", "dtb_plan_destroy", "dtb_status_string"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(dtb.EXPORTS)


def test_status_strings():
    for code, name in dtb.STATUS.items():
        assert dtb.status_string(code) == name
    assert dtb.status_string(-99) == "DTB_ERR_UNKNOWN"


def _plan_rc(rows, cols, pitch, dtype, opts=None, out=True):
    lib = dtb.load()
    h = ctypes.c_void_p()
    o = ctypes.byref(opts) if opts is not None else None
    return lib.dtb_plan(ctypes.byref(h) if out else None, rows, cols, pitch, dtype, 0, o)


@pytest.mark.parametrize("args", [(0, 5, 7, 0), (5, 0, 7, 0), (5, 5, 6, 0), (5, 5, 7, 2), (-1, 5, 7, 1)])
def test_plan_rejects_bad_shape(args):
    assert _plan_rc(*args) == -1


def test_plan_rejects_null_out_and_bad_options():
    assert _plan_rc(5, 5, 7, 0, out=False) == -1
    for field, value in [("path", 9), ("ghost_k", -1), ("exact", 2), ("debug_flags", 16), ("max_wg", -3), ("tune", 2), ("waves", 6)]:
        o = dtb.PlanOpts()
        setattr(o, field, value)
        assert _plan_rc(5, 5, 7, 0, o) == -1, field


def test_run_rejects_bad_arguments():
    lib = dtb.load()
    c = (ctypes.c_double * 5)(0.2, 0.2, 0.2, 0.2, 0.2)
    g = dtb.Grid(0, 5, 5, 7)
    assert lib.dtb_run(ctypes.byref(g), c, 3, 0, None) == -1          # NULL data
    g = dtb.Grid(0x1000, 5, 5, 7)
    assert lib.dtb_run(ctypes.byref(g), c, -1, 0, None) == -1         # T < 0
    assert lib.dtb_run(None, c, 3, 0, None) == -1
    assert lib.dtb_run(ctypes.byref(g), None, 3, 0, None) == -1
    assert lib.dtb_run(ctypes.byref(g), c, 3, 5, None) == -1          # dtype
    g = dtb.Grid(0x1000, 5, 5, 6)
    assert lib.dtb_run(ctypes.byref(g), c, 3, 0, None) == -1          # pitch
    g = dtb.Grid(0x1000, 5, 5, 7)
    assert lib.dtb_run(ctypes.byref(g), c, 0, 0, None) == 0           # T == 0: no-op, no HIP call
    assert lib.dtb_run_batched(None, -1, None) == -1
    assert lib.dtb_run_batched(None, 0, None) == 0
    p = (dtb.Problem * 1)()
    p[0].grid = dtb.Grid(0, 5, 5, 7)
    assert lib.dtb_run_batched(p, 1, None) == -1
    assert lib.dtb_run_plan(None, ctypes.byref(g), c, 1, None) == -1
    assert lib.dtb_plan_check(None, None) == -1
    lib.dtb_plan_destroy(None)


def test_plan_rejects_missing_instances_before_any_hip_call():
    """Tile instances that do not exist are DTB_ERR_UNSUPPORTED, decided on the host."""
    cases = [(dtb.F32, dict(rows_per_lane=12)),                      # 4-column tile is FP64 only
             (dtb.F32, dict(waves=4)),                               # half-height workgroups: FP64 only
             (dtb.F64, dict(waves=4, rows_per_lane=16)),             # ... and 24 rows per lane only
             (dtb.F64, dict(waves=4, path=dtb.PATH_SWEEP)),          # ... and the resident path only
             (dtb.F64, dict(rows_per_lane=28)),                      # 28 rows: FP32 only
             (dtb.F64, dict(rows_per_lane=10))]
    for dtype, fields in cases:
        o = dtb.PlanOpts()
        for k, v in fields.items():
            setattr(o, k, v)
        assert _plan_rc(64, 64, 66, dtype, o) == -2, (dtype, fields)


def test_noalloc_refuses_before_any_hip_call():
    """dtb_run_noalloc: invalid arguments and grids larger than its fixed area are refused on the host."""
    lib = dtb.load()
    c = (ctypes.c_double * 5)(0.2, 0.2, 0.2, 0.2, 0.2)
    assert lib.dtb_run_noalloc(None, c, 3, 0, None, None) == -1
    g = dtb.Grid(0, 5, 5, 7)
    assert lib.dtb_run_noalloc(ctypes.byref(g), c, 3, 0, None, None) == -1          # NULL data
    g = dtb.Grid(0x1000, 5, 5, 6)
    assert lib.dtb_run_noalloc(ctypes.byref(g), c, 3, 0, None, None) == -1          # pitch
    g = dtb.Grid(0x1000, 5, 5, 7)
    assert lib.dtb_run_noalloc(ctypes.byref(g), c, -1, 0, None, None) == -1         # T
    assert lib.dtb_run_noalloc(ctypes.byref(g), c, 3, 7, None, None) == -1          # dtype
    assert lib.dtb_run_noalloc(ctypes.byref(g), c, 0, 0, None, None) == 0           # T == 0: nothing to do
    # 1534^2 FP64 (storage 1536 x 1536 = 18 MiB) is the largest square grid that fits; 1535^2 does not.
    g = dtb.Grid(0x1000, 1535, 1535, 1537)
    assert lib.dtb_run_noalloc(ctypes.byref(g), c, 3, 0, None, None) == -2
    g = dtb.Grid(0x1000, 2171, 2171, 2173)                                          # FP32: 2170^2 is the largest
    assert lib.dtb_run_noalloc(ctypes.byref(g), c, 3, 1, None, None) == -2


def test_plan_rejects_bad_sync_and_overlapped_options():
    o = dtb.PlanOpts()
    o.sync = 2
    assert _plan_rc(64, 64, 66, 0, o) == -1
    for fields in (dict(sync=1, path=dtb.PATH_SWEEP), dict(sync=1, path=dtb.PATH_OVERLAPPED),
                   dict(path=dtb.PATH_OVERLAPPED, rows_per_lane=16), dict(path=dtb.PATH_OVERLAPPED, waves=4)):
        o = dtb.PlanOpts()
        for k, v in fields.items():
            setattr(o, k, v)
        assert _plan_rc(64, 64, 66, 0, o) == -2, fields


def test_plan_box_stencil_options_checked_on_the_host():
    """stencil must be 0, 5, 7 or 9; the box has no overlapped path, no half-height or grid-barrier variant, and
    only its own register tiles (FP64 8 rows per lane, FP32 16)."""
    for bad in (1, 8, 25, -5):  # 7 (j3d7pt) is a 3-D plan: refused as unsupported below
        o = dtb.PlanOpts()
        o.stencil = bad
        assert _plan_rc(64, 64, 66, 0, o) == -1, bad
    cases = [(dtb.F64, dict(path=dtb.PATH_OVERLAPPED)),
             (dtb.F64, dict(waves=4)),
             (dtb.F64, dict(sync=1)),
             (dtb.F64, dict(rows_per_lane=12)),     # the 5-point FP64 tile, not a box tile
             (dtb.F64, dict(rows_per_lane=16)),     # the FP32 box height
             (dtb.F32, dict(rows_per_lane=8)),      # the FP64 box height
             (dtb.F32, dict(rows_per_lane=24, path=dtb.PATH_SWEEP))]
    for dtype, fields in cases:
        o = dtb.PlanOpts()
        o.stencil = 9
        for k, v in fields.items():
            setattr(o, k, v)
        assert _plan_rc(64, 64, 66, dtype, o) == -2, (dtype, fields)


def test_box_plan_takes_nine_coefficients():
    with pytest.raises(ValueError):
        dtb._coeffs([0.2] * 5, 9)
    with pytest.raises(ValueError):
        dtb._coeffs([0.1] * 9, 5)
    assert len(dtb._coeffs([0.1] * 9, 9)) == 9


def test_plan3d_rejects_bad_shapes_and_options_before_any_hip_call():
    lib = dtb.load()
    h = ctypes.c_void_p()

    def rc(depth, rows, cols, pitch, pp, dtype=0, **fields):
        o = dtb.PlanOpts()
        for k, v in fields.items():
            setattr(o, k, v)
        return lib.dtb_plan3d(ctypes.byref(h), depth, rows, cols, pitch, pp, dtype, ctypes.byref(o))

    assert lib.dtb_plan3d(None, 4, 4, 4, 6, 36, 0, None) == -1
    for bad in [(0, 4, 4, 6, 36), (4, 0, 4, 6, 36), (4, 4, 0, 6, 36), (4, 4, 4, 5, 36), (4, 4, 4, 6, 35)]:
        assert rc(*bad) == -1, bad
    assert rc(4, 4, 4, 6, 36, dtype=3) == -1
    assert rc(4, 4, 4, 6, 36, stencil=9) == -1            # a 3-D plan is j3d7pt
    for fields in (dict(path=dtb.PATH_RESIDENT), dict(path=dtb.PATH_SWEEP), dict(ghost_k=4), dict(sync=1),
                   dict(tune=1), dict(waves=4), dict(debug_flags=dtb.DEBUG_POISON)):
        assert rc(4, 4, 4, 6, 36, **fields) == -2, fields
    # columns per lane: an instance's (FP64 2; FP32 4 or 3), else unsupported; negative: invalid
    assert rc(4, 4, 4, 6, 36, cols_per_lane=-1) == -1
    for dtype, fields in ((dtb.F64, dict(cols_per_lane=3)), (dtb.F64, dict(cols_per_lane=4)),
                          (dtb.F32, dict(cols_per_lane=2)), (dtb.F32, dict(cols_per_lane=5)),
                          (dtb.F32, dict(cols_per_lane=3, rows_per_lane=8)),
                          (dtb.F64, dict(cols_per_lane=2, path=dtb.PATH_STEP))):
        assert rc(4, 4, 4, 6, 36, dtype=dtype, **fields) == -2, (dtype, fields)
    # and a 2-D plan refuses the 3-D stencil and path, and the 3-D column choice
    assert _plan_rc(64, 64, 66, 0, _opts(stencil=7)) == -2
    assert _plan_rc(64, 64, 66, 0, _opts(path=dtb.PATH_STREAM3D)) == -2
    assert _plan_rc(64, 64, 66, 0, _opts(cols_per_lane=2)) == -2
    assert _plan_rc(64, 64, 66, 0, _opts(cols_per_lane=-2)) == -1


def _opts(**fields):
    o = dtb.PlanOpts()
    for k, v in fields.items():
        setattr(o, k, v)
    return o


def test_run3d_rejects_bad_arguments():
    lib = dtb.load()
    c = (ctypes.c_double * 7)(*([1.0 / 7] * 7))
    g = dtb.Grid3(0x1000, 4, 4, 4, 6, 36)
    assert lib.dtb_run3d_plan(None, ctypes.byref(g), c, 1, None) == -1
    assert lib.dtb_run3d_plan(None, None, c, 1, None) == -1
