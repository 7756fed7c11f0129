"""ctypes binding for libdtb (include/dtb.h): argument marshalling only.

Every computation happens in the HIP kernels of libdtb.so.  If the library is
missing this module raises; there is no other code path.

Grids are torch tensors on a ROCm device, shape (rows + 2, pitch) --
interior [1:rows+1, 1:cols+1], one-cell Dirichlet halo -- of dtype float64
(DTB_F64) or float32 (DTB_F32).  ``cols`` defaults to ``pitch - 2``.
Coefficients are (c, n, s, e, w).  Work is enqueued on torch's current
stream unless a stream is given.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdtb.so")

F64, F32 = 0, 1
DEBUG_TINY_SPIN, DEBUG_POISON, DEBUG_TIMING, DEBUG_DIRECT_XCHG = 1, 2, 4, 8
PATH_AUTO, PATH_STEP, PATH_RESIDENT, PATH_SWEEP, PATH_OVERLAPPED, PATH_STREAM3D = 0, 1, 2, 3, 4, 5
SYNC_NEIGHBOURS, SYNC_GRID_BARRIER = 0, 1
STATUS = {0: "DTB_OK", -1: "DTB_ERR_INVALID_ARG", -2: "DTB_ERR_UNSUPPORTED", -3: "DTB_ERR_NOT_CORESIDENT",
          -4: "DTB_ERR_OUT_OF_MEMORY", -5: "DTB_ERR_HIP", -6: "DTB_ERR_TIMEOUT", -7: "DTB_ERR_NOT_PLANNED",
          -8: "DTB_ERR_MISMATCH"}
DESCRIBE_FIELDS = ("path", "workgroups", "ghost_k", "depth_D", "ext_rows", "ext_cols", "tiles_rows",
                   "tiles_cols", "rows_per_lane", "cols_per_lane", "big_tiles", "exact", "waves", "sync",
                   "stencil")
STENCIL_J2D5PT, STENCIL_BOX = 5, 9
TEST_MAX_NEIGHBOURS = 24
TIMING_SLOTS = 11
TEST_LAYOUT_STRIDE = 8 + TEST_MAX_NEIGHBOURS


class DtbError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}" if what else STATUS.get(status, str(status)))


class Grid(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("pitch", ctypes.c_int64)]


class Grid3(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("depth", ctypes.c_int64), ("rows", ctypes.c_int64),
                ("cols", ctypes.c_int64), ("pitch", ctypes.c_int64), ("plane_pitch", ctypes.c_int64)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("ghost_k", ctypes.c_int32), ("depth_D", ctypes.c_int32),
                ("rows_per_lane", ctypes.c_int32), ("max_wg", ctypes.c_int32), ("exact", ctypes.c_int32),
                ("debug_flags", ctypes.c_int32), ("tune", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("sync", ctypes.c_int32), ("stencil", ctypes.c_int32), ("cols_per_lane", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("grid", Grid), ("coeffs", ctypes.c_double * 5), ("T", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


# Every symbol include/dtb.h and include/dtb_testing.h declare.
EXPORTS = ("dtb_plan", "dtb_run_plan", "dtb_run", "dtb_run_batched", "dtb_plan_check", "dtb_plan_describe",
           "dtb_plan_destroy", "dtb_cache_clear", "dtb_status_string", "dtb_test_layout", "dtb_test_sweep",
           "dtb_batch_check", "dtb_test_batch", "dtb_plan_timing", "dtb_probe", "dtb_run_noalloc", "dtb_plan3d",
           "dtb_run3d_plan", "dtb_test_split3", "dtb_test_zblock", "dtb_test_cols3")
TEST_SWEEP_STRIDE = 17 + TEST_MAX_NEIGHBOURS

_lib = None


def load():
    """Load libdtb.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: run __graft_entry__.build() (or python -m paper_2306_03336_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.dtb_plan.restype = ctypes.c_int
    lib.dtb_plan.argtypes = [ctypes.POINTER(P), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                             ctypes.c_int64, ctypes.POINTER(PlanOpts)]
    lib.dtb_run_plan.restype = ctypes.c_int
    lib.dtb_run_plan.argtypes = [P, ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_double), ctypes.c_int64, P]
    lib.dtb_plan3d.restype = ctypes.c_int
    lib.dtb_plan3d.argtypes = [ctypes.POINTER(P), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_int64, ctypes.c_int, ctypes.POINTER(PlanOpts)]
    lib.dtb_run3d_plan.restype = ctypes.c_int
    lib.dtb_run3d_plan.argtypes = [P, ctypes.POINTER(Grid3), ctypes.POINTER(ctypes.c_double), ctypes.c_int64, P]
    lib.dtb_test_split3.restype = ctypes.c_int32
    lib.dtb_test_split3.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.c_int32]
    lib.dtb_test_zblock.restype = ctypes.c_int32
    lib.dtb_test_zblock.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
    lib.dtb_test_cols3.restype = ctypes.c_int32
    lib.dtb_test_cols3.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
    lib.dtb_run.restype = ctypes.c_int
    lib.dtb_run.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int, P]
    lib.dtb_run_batched.restype = ctypes.c_int
    lib.dtb_run_batched.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32, P]
    lib.dtb_plan_check.restype = ctypes.c_int
    lib.dtb_plan_check.argtypes = [P, P]
    lib.dtb_plan_describe.restype = ctypes.c_int
    lib.dtb_plan_describe.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
    lib.dtb_plan_destroy.restype = None
    lib.dtb_plan_destroy.argtypes = [P]
    lib.dtb_cache_clear.restype = None
    lib.dtb_cache_clear.argtypes = []
    lib.dtb_status_string.restype = ctypes.c_char_p
    lib.dtb_status_string.argtypes = [ctypes.c_int]
    lib.dtb_test_layout.restype = ctypes.c_int32
    lib.dtb_test_layout.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    lib.dtb_plan_timing.restype = ctypes.c_int
    lib.dtb_plan_timing.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32, P]
    lib.dtb_batch_check.restype = ctypes.c_int
    lib.dtb_batch_check.argtypes = [P]
    I64P, I32P = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
    lib.dtb_test_batch.restype = ctypes.c_int32
    lib.dtb_test_batch.argtypes = [ctypes.c_int32, I64P, I64P, I32P, I64P, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, I32P, I32P, ctypes.c_int32, I64P]
    lib.dtb_test_sweep.restype = ctypes.c_int32
    lib.dtb_test_sweep.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    lib.dtb_run_noalloc.restype = ctypes.c_int
    lib.dtb_run_noalloc.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                                    ctypes.c_int, P, P]
    lib.dtb_probe.restype = ctypes.c_int
    lib.dtb_probe.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P,
                              ctypes.POINTER(ctypes.c_double)]
    _lib = lib
    return lib


def status_string(s: int) -> str:
    return load().dtb_status_string(int(s)).decode()


def _check(rc: int, what: str):
    if rc != 0:
        raise DtbError(rc, what)


def _coeffs(coeffs, n: int = 5):
    c = [float(x) for x in coeffs]
    if len(c) != n:
        raise ValueError("five coefficients (c, n, s, e, w) are required" if n == 5 else
                         "nine coefficients (sw, s, se, w, c, e, nw, n, ne) are required")
    return (ctypes.c_double * n)(*c)


def _dtype_of(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _grid(t, cols=None) -> Grid:
    if t.dim() != 2 or not t.is_cuda:
        raise ValueError("grid must be a 2-D device tensor of shape (rows + 2, pitch)")
    if t.stride(1) != 1:
        raise ValueError("grid rows must be contiguous")
    rows = t.shape[0] - 2
    pitch = t.stride(0)
    cols = t.shape[1] - 2 if cols is None else int(cols)
    return Grid(t.data_ptr(), rows, cols, pitch)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """An explicit plan (dtb_plan / dtb_run_plan / dtb_plan_destroy)."""

    def __init__(self, rows: int, cols: int, pitch: int, dtype: int, T_hint: int = 0, path: int = PATH_AUTO,
                 ghost_k: int = 0, depth_D: int = 0, rows_per_lane: int = 0, max_wg: int = 0, exact: bool = False,
                 tune: bool = False, debug: int = 0, waves: int = 0, sync: int = 0, stencil: int = 5):
        lib = load()
        self._h = ctypes.c_void_p()
        opts = PlanOpts(path, ghost_k, depth_D, rows_per_lane, max_wg, 1 if exact else 0, debug, 1 if tune else 0,
                        waves, sync, stencil)
        _check(lib.dtb_plan(ctypes.byref(self._h), rows, cols, pitch, dtype, T_hint, ctypes.byref(opts)), "dtb_plan")
        self.rows, self.cols, self.pitch, self.dtype = rows, cols, pitch, dtype
        self.stencil = 9 if stencil == 9 else 5

    def run(self, grid, coeffs, T: int, stream=None, cols=None):
        """Advance `grid` T steps in place: five coefficients (c, n, s, e, w), or nine (sw, s, se, w, c, e, nw,
        n, ne) for a plan made with stencil=9."""
        g = _grid(grid, cols)
        _check(load().dtb_run_plan(self._h, ctypes.byref(g), _coeffs(coeffs, self.stencil), int(T),
                                   _stream(stream)), "dtb_run_plan")

    def check(self, stream=None):
        _check(load().dtb_plan_check(self._h, _stream(stream)), "dtb_plan_check")

    def timing(self, stream=None):
        """Per-workgroup phase clocks (DTB_DEBUG_TIMING plans): list of dicts, times in microseconds."""
        n = self.describe()["workgroups"]
        m = TIMING_SLOTS
        buf = (ctypes.c_uint64 * (m * n))()
        _check(load().dtb_plan_timing(self._h, buf, m * n, _stream(stream)), "dtb_plan_timing")
        names = ("steps", "publish", "wait", "ghost")
        out = []
        for i in range(n):
            v = buf[m * i:m * i + m]
            d = {k: v[j] / 100.0 for j, k in enumerate(names)}  # 100 MHz ticks -> us
            d["exchanges"] = int(v[4])
            d["total"] = v[5] / 100.0
            d["stage_out"] = v[6] / 100.0
            d["stage_in"] = v[7] / 100.0
            d["load"] = v[8] / 100.0
            d["store"] = v[9] / 100.0
            d["barrier"] = v[10] / 100.0
            out.append(d)
        return out

    def describe(self) -> dict:
        vals = (ctypes.c_int64 * len(DESCRIBE_FIELDS))()
        _check(load().dtb_plan_describe(self._h, vals, len(DESCRIBE_FIELDS)), "dtb_plan_describe")
        return dict(zip(DESCRIBE_FIELDS, (int(v) for v in vals)))

    def destroy(self):
        if self._h:
            load().dtb_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _grid3(t, cols=None) -> Grid3:
    if t.dim() != 3 or not t.is_cuda:
        raise ValueError("grid must be a 3-D device tensor of shape (depth + 2, rows + 2, pitch)")
    if t.stride(2) != 1 or t.stride(1) < t.shape[2] or t.stride(0) < t.shape[1] * t.stride(1):
        raise ValueError("grid rows must be contiguous and planes must not overlap")
    cols = t.shape[2] - 2 if cols is None else int(cols)
    return Grid3(t.data_ptr(), t.shape[0] - 2, t.shape[1] - 2, cols, t.stride(1), t.stride(0))


class Plan3D(Plan):
    """An explicit j3d7pt plan (dtb_plan3d / dtb_run3d_plan / dtb_plan_destroy)."""

    def __init__(self, depth: int, rows: int, cols: int, pitch: int, plane_pitch: int, dtype: int,
                 path: int = PATH_AUTO, ghost_k: int = 0, depth_D: int = 0, rows_per_lane: int = 0, max_wg: int = 0,
                 exact: bool = False, cols_per_lane: int = 0):
        lib = load()
        self._h = ctypes.c_void_p()
        opts = PlanOpts(path, ghost_k, depth_D, rows_per_lane, max_wg, 1 if exact else 0, 0, 0, 0, 0, 7,
                        cols_per_lane)
        _check(lib.dtb_plan3d(ctypes.byref(self._h), depth, rows, cols, pitch, plane_pitch, dtype, ctypes.byref(opts)),
               "dtb_plan3d")
        self.rows, self.cols, self.pitch, self.dtype = rows, cols, pitch, dtype
        self.depth, self.plane_pitch, self.stencil = depth, plane_pitch, 7

    def run(self, grid, coeffs, T: int, stream=None, cols=None):
        """Advance the 3-D `grid` T steps in place: seven coefficients (c, n, s, e, w, t, b)."""
        g = _grid3(grid, cols)
        c = [float(x) for x in coeffs]
        if len(c) != 7:
            raise ValueError("seven coefficients (c, n, s, e, w, t, b) are required")
        _check(load().dtb_run3d_plan(self._h, ctypes.byref(g), (ctypes.c_double * 7)(*c), int(T), _stream(stream)),
               "dtb_run3d_plan")


def plan3d_for(grid, cols=None, **opts) -> Plan3D:
    g = _grid3(grid, cols)
    return Plan3D(g.depth, g.rows, g.cols, g.pitch, g.plane_pitch, _dtype_of(grid), **opts)


def plan_for(grid, T_hint: int = 0, cols=None, **opts) -> Plan:
    g = _grid(grid, cols)
    return Plan(g.rows, g.cols, g.pitch, _dtype_of(grid), T_hint, **opts)


def run(grid, coeffs, T: int, stream=None, cols=None):
    """dtb_run: advance `grid` T steps in place with a cached default plan."""
    g = _grid(grid, cols)
    _check(load().dtb_run(ctypes.byref(g), _coeffs(coeffs), int(T), _dtype_of(grid), _stream(stream)), "dtb_run")


def run_noalloc(grid, coeffs, T: int, err_flag=None, stream=None, cols=None):
    """dtb_run_noalloc: as run(), with no allocation (resident grids that fit the library's fixed area).
    err_flag: None or a one-element int32 device tensor into which a timed-out wait ORs a nonzero value."""
    g = _grid(grid, cols)
    errp = None if err_flag is None else ctypes.c_void_p(err_flag.data_ptr())
    _check(load().dtb_run_noalloc(ctypes.byref(g), _coeffs(coeffs), int(T), _dtype_of(grid), errp,
                                  _stream(stream)), "dtb_run_noalloc")


def run_batched(problems, stream=None):
    """dtb_run_batched over [(grid, coeffs, T), ...]."""
    arr = (Problem * len(problems))()
    for i, (grid, coeffs, T) in enumerate(problems):
        arr[i].grid = _grid(grid)
        arr[i].coeffs = _coeffs(coeffs)
        arr[i].T = int(T)
        arr[i].dtype = _dtype_of(grid)
    _check(load().dtb_run_batched(arr, len(problems), _stream(stream)), "dtb_run_batched")


def batch_check(stream=None):
    """dtb_batch_check: wait for the stream, raise if a batched launch recorded a failure."""
    _check(load().dtb_batch_check(_stream(stream)), "dtb_batch_check")


PROBE_LDS_READ, PROBE_LDS_WRITE, PROBE_COPY, PROBE_BARRIER, PROBE_FLAGS = 0, 1, 2, 3, 4


def probe(kind: int, size: int = 0, iters: int = 1, nwg: int = 0, stream=None):
    """dtb_probe: run one micro-benchmark; returns (milliseconds, work) -- work is bytes moved
    (LDS, copy) or the number of barriers / exchange points."""
    out = (ctypes.c_double * 2)()
    _check(load().dtb_probe(int(kind), int(size), int(iters), int(nwg), _stream(stream), out), "dtb_probe")
    return out[0], out[1]


def cache_clear():
    load().dtb_cache_clear()


def test_layout(rows: int, cols: int, rows_per_lane: int, cols_per_lane: int, waves: int, k: int,
                n_xcd: int = 8, max_wg: int = 4096):
    """Planner layout without a GPU: list of dicts per workgroup in launch order (or None)."""
    buf = (ctypes.c_int32 * (max_wg * TEST_LAYOUT_STRIDE))()
    n = load().dtb_test_layout(rows, cols, rows_per_lane, cols_per_lane, waves, k, n_xcd, buf, max_wg)
    if n < 0 or n > max_wg:
        return None
    out = []
    for i in range(n):
        o = buf[i * TEST_LAYOUT_STRIDE:(i + 1) * TEST_LAYOUT_STRIDE]
        out.append(dict(ext_r0=o[0], ext_c0=o[1], own_r0=o[2], own_r1=o[3], own_c0=o[4], own_c1=o[5],
                        nb=[x for x in o[7:7 + o[6]]], narrow_rows=bool(o[7 + TEST_MAX_NEIGHBOURS] & 1),
                        narrow_cols=bool(o[7 + TEST_MAX_NEIGHBOURS] & 2)))
    return out


def test_split3(n: int, E: int, K: int):
    """3-D streaming planner's split of one axis, without a GPU: list of (e0, own0, own1), or None."""
    lib = load()
    m = lib.dtb_test_split3(n, E, K, None, 0)
    if m < 0:
        return None
    buf = (ctypes.c_int32 * (3 * m))()
    assert lib.dtb_test_split3(n, E, K, buf, m) == m
    return [tuple(buf[3 * i:3 * i + 3]) for i in range(m)]


def test_zblock(ntiles: int, ext_rows: int, ext_cols: int, K: int, elem_bytes: int, depth: int,
                interior_cells: int, n_cu: int = 256):
    """The z-block height the 3-D streaming planner picks, without a GPU (or None for invalid arguments)."""
    z = load().dtb_test_zblock(ntiles, ext_rows, ext_cols, K, elem_bytes, depth, interior_cells, n_cu)
    return None if z < 0 else z


def test_cols3(dtype: int, cols: int, K: int = 3):
    """The columns per lane of the 3-D streaming instance the planner picks, without a GPU (None: invalid)."""
    c = load().dtb_test_cols3(dtype, cols, K)
    return None if c < 0 else c


def test_sweep(rows: int, cols: int, rows_per_lane: int, cols_per_lane: int, waves: int, k: int, D: int,
               max_wg: int, n_xcd: int = 8):
    """Sweep planner without a GPU: list of big tiles, each a list of per-slot dicts (or None)."""
    lib = load()
    n = lib.dtb_test_sweep(rows, cols, rows_per_lane, cols_per_lane, waves, k, D, max_wg, n_xcd, None, 0)
    if n < 0:
        return None
    buf = (ctypes.c_int32 * (n * TEST_SWEEP_STRIDE))()
    n2 = lib.dtb_test_sweep(rows, cols, rows_per_lane, cols_per_lane, waves, k, D, max_wg, n_xcd, buf, n)
    assert n2 == n
    tiles = {}
    for i in range(n):
        o = buf[i * TEST_SWEEP_STRIDE:(i + 1) * TEST_SWEEP_STRIDE]
        tiles.setdefault(o[0], []).append(dict(
            nwg=o[1], ext_r0=o[2], ext_c0=o[3], own_r0=o[4], own_r1=o[5], own_c0=o[6], own_c1=o[7],
            cr=(o[8], o[9], o[10], o[11]), st=(o[12], o[13], o[14], o[15]), nb=[x for x in o[17:17 + o[16]]]))
    return [tiles[t] for t in sorted(tiles)]


TEST_BATCH_STRIDE = 13


def test_batch(shapes, r64: int = 0, r32: int = 0, n_slots: int = 256):
    """Batch planner without a GPU.  shapes: [(rows, cols, dtype, T), ...].  r64 = r32 = 0: the register-tile
    instances the batched kernel carries; else one instance per precision (FP64 2 x r64, FP32 4 x r32).
    Returns (jobs, slot_lists) or None; jobs are dicts in global order, slot_lists[s] = [(job, member), ...]."""
    n = len(shapes)
    I64 = ctypes.c_int64 * n
    rows = I64(*[s[0] for s in shapes])
    cols = I64(*[s[1] for s in shapes])
    dt = (ctypes.c_int32 * n)(*[s[2] for s in shapes])
    T = I64(*[s[3] for s in shapes])
    jobs = (ctypes.c_int32 * (n * TEST_BATCH_STRIDE))()
    cap = n_slots + 1 + 2 * n * n_slots
    lists = (ctypes.c_int32 * cap)()
    info = (ctypes.c_int64 * 2)()
    rc = load().dtb_test_batch(n, rows, cols, dt, T, r64, r32, n_slots, jobs, lists, cap, info)
    if rc < 0:
        return None
    test_batch.last_info = {"makespan_us": int(info[0]), "spin_limit": int(info[1])}
    keys = ("prob", "g", "sweep", "ntiles", "D", "nrounds", "flag_base", "table_off", "start", "dur", "k", "R", "C")
    st = TEST_BATCH_STRIDE
    jl = [dict(zip(keys, jobs[j * st:(j + 1) * st])) for j in range(rc)]
    off = lists[:n_slots + 1]
    pairs = lists[n_slots + 1:n_slots + 1 + 2 * off[-1]]
    sl = [[(pairs[2 * i], pairs[2 * i + 1]) for i in range(off[s], off[s + 1])] for s in range(n_slots)]
    return jl, sl
