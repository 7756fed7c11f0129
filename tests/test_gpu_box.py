"""GPU parity of the 3 x 3 box stencil (j2d9pt): libdtb plans made with stencil=9, through the C ABI,
against the box oracle (oracle/j2d9pt_oracle.c).

Exact mode (separately rounded products summed sw, s, se, w, c, e, nw, n, ne) must match the oracle bit for
bit, FP64 against the FP64 oracle and FP32 against the FP32 oracle, on the resident path, the tile-serial
sweep and the one-step path.  The default fused chain must stay within 1e-13 relative max-norm of the FP64
oracle, and FP32 within its a priori bound.  Every case prints its parameters before it touches the GPU.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2306_03336_amd import dtb, inputs
from record import oracle_in_chunks, record

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_F64 = 1e-13
U_F32 = 2.0 ** -24


def f32_bound9(T):
    """A priori relative max-norm bound of FP32 against the FP64 oracle for non-negative weights summing to
    1: at most nine roundings per cell per step, one of each input cell and of each weight (acting once per
    step), doubled for safety: 2 (10 T + 1) u."""
    return 2 * (10 * T + 1) * U_F32


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _dev(u):
    return torch.from_numpy(np.ascontiguousarray(u)).to("cuda")


def _random_halo(u, rng, rows, cols):
    """A halo that changes along every side, corners included (the box reads them)."""
    u[0, :cols + 2] = rng.uniform(-1, 2, cols + 2)
    u[rows + 1, :cols + 2] = rng.uniform(-1, 2, cols + 2)
    u[:, 0] = rng.uniform(-1, 2, rows + 2)
    u[:, cols + 1] = rng.uniform(-1, 2, rows + 2)
    return u


def _run_plan(u, coeffs, T, dtype=np.float64, cols=None, **opts):
    g = _dev(u.astype(dtype))
    plan = dtb.plan_for(g, T, cols=cols, stencil=9, **opts)
    plan.run(g, coeffs, T, cols=cols)
    plan.check()
    desc = plan.describe()
    out = g.cpu().numpy()
    plan.destroy()
    return out, desc


def _skip_if_spilling(e, i, what):
    # A variant whose registers spill is never chosen: the planner refuses it (DTB_ERR_NOT_CORESIDENT).  The
    # refusal depends on the shape only, so it comes at the first case or not at all.
    assert i == 0 and e.status == -3, (what, e)
    pytest.skip(f"{what}: the kernel variant for this shape spills registers; the planner refuses it")


SHAPES = [(1, 1), (1, 37), (45, 1), (3, 200), (64, 256), (127, 131), (256, 256), (200, 300), (70, 130),
          (129, 257), (600, 700)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_box_exact_f64_bitwise(shape):
    rows, cols = shape
    rng = np.random.default_rng(rows * 1000 + cols + 9)
    coeffs = inputs.box_weights(rng)
    u_var = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols)
    u_const = inputs.uniform_grid(rows, cols, rng, halo=0.625)
    for i, ((k, T), u) in enumerate(zip([(1, 3), (2, 7), (4, 4), (5, 23), (8, 37), (16, 9), (3, 17), (8, 40)],
                                        [u_var] * 6 + [u_const] * 2)):
        _say("box exact f64", rows, cols, "k", k, "T", T)
        try:
            got, desc = _run_plan(u, coeffs, T, path=dtb.PATH_RESIDENT, ghost_k=k, exact=True)
        except dtb.DtbError as e:
            _skip_if_spilling(e, i, f"box exact FP64 {rows}x{cols}")
        assert desc["path"] == dtb.PATH_RESIDENT and desc["exact"] == 1 and desc["stencil"] == 9, desc
        assert desc["rows_per_lane"] == 8 and desc["cols_per_lane"] == 4, desc
        ref = oracle.j2d9pt_f64(u, coeffs, T)
        assert np.array_equal(got, ref), (rows, cols, k, T, float(np.max(np.abs(got - ref))))


@pytest.mark.parametrize("shape", [(1, 1), (40, 1), (2, 300), (131, 127), (256, 256), (90, 520), (517, 389)],
                         ids=lambda s: f"{s[0]}x{s[1]}")
def test_box_exact_f32_bitwise(shape):
    rows, cols = shape
    rng = np.random.default_rng(rows * 7 + cols + 99)
    # strongly asymmetric weights: drive cells toward subnormals
    coeffs = (0.01, 0.3, 0.002, 0.05, 0.04, 0.4, 0.003, 0.005, 0.19)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols).astype(np.float32)
    for i, (k, T) in enumerate([(2, 5), (6, 40), (8, 200), (11, 60), (12, 50)]):
        _say("box exact f32", rows, cols, "k", k, "T", T)
        try:
            got, desc = _run_plan(u, coeffs, T, dtype=np.float32, path=dtb.PATH_RESIDENT, ghost_k=k, exact=True)
        except dtb.DtbError as e:
            _skip_if_spilling(e, i, f"box exact FP32 {rows}x{cols}")
        assert desc["rows_per_lane"] == 16 and desc["stencil"] == 9, desc
        ref = oracle.j2d9pt_f32(u, coeffs, T)
        assert np.array_equal(got, ref), (rows, cols, k, T)


@pytest.mark.parametrize("case", [
    # rows, cols, max_wg, k, D, T
    (600, 700, 8, 4, 16, 37),      # several big tiles, T not a multiple of D, odd rounds
    (600, 700, 8, 3, 10, 40),      # even rounds
    (1000, 333, 6, 5, 12, 25),
    (300, 1100, 12, 6, 20, 61),
    (257, 129, 4, 2, 7, 9),
    (130, 900, 8, 4, 9, 5),        # T < D: one short round
], ids=lambda c: "x".join(map(str, c)))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_box_sweep_exact_bitwise(case, dtype):
    rows, cols, max_wg, k, D, T = case
    npd = np.float64 if dtype == "f64" else np.float32
    ref_fn = oracle.j2d9pt_f64 if dtype == "f64" else oracle.j2d9pt_f32
    rng = np.random.default_rng(rows + 7 * cols + T + 9)
    coeffs = inputs.box_weights(rng)
    u_var = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols).astype(npd)
    u_const = inputs.uniform_grid(rows, cols, rng, halo=0.375).astype(npd)
    if dtype == "f32":
        max_wg = max(1, max_wg // 2)  # the FP32 box tile (128 x 256) is twice as tall: half the workgroups
        # give at least two big tiles in every case, as the FP64 cases have
    for i, u in enumerate((u_var, u_const)):
        _say("box sweep", dtype, case, "max_wg", max_wg)
        try:
            got, desc = _run_plan(u, coeffs, T, dtype=npd, path=dtb.PATH_SWEEP, ghost_k=k, depth_D=D,
                                  max_wg=max_wg, exact=True)
        except dtb.DtbError as e:
            _skip_if_spilling(e, i, f"box sweep {dtype} {rows}x{cols}")
        assert desc["path"] == dtb.PATH_SWEEP and desc["depth_D"] == D and desc["big_tiles"] >= 2, desc
        ref = ref_fn(u, coeffs, T)
        assert np.array_equal(got, ref), (case, float(np.max(np.abs(got.astype(float) - ref))))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape_pitch", [(1, 1, 4), (64, 1, 4), (33, 130, 132), (129, 254, 256), (129, 255, 260),
                                         (300, 700, 703)],
                         ids=lambda s: "x".join(map(str, s)))
def test_box_step_path_bitwise(dtype, shape_pitch):
    """The one-step baseline of the box, exact mode, against the oracle bit for bit; both of its access widths
    (16-byte groups when the pitch allows, single elements otherwise); and its fused chain equals the DTB
    kernels' fused chain bit for bit."""
    rows, cols, pitch = shape_pitch
    npd = np.float64 if dtype == "f64" else np.float32
    ref_fn = oracle.j2d9pt_f64 if dtype == "f64" else oracle.j2d9pt_f32
    rng = np.random.default_rng(rows + cols + pitch)
    coeffs = inputs.box_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng, pitch=pitch), rng, rows, cols).astype(npd)
    T = 7
    _say("box step", dtype, rows, cols, pitch)
    got, desc = _run_plan(u, coeffs, T, dtype=npd, cols=cols, path=dtb.PATH_STEP, exact=True)
    assert desc["path"] == dtb.PATH_STEP
    ref = ref_fn(u, coeffs, T, cols=cols)
    assert np.array_equal(got, ref), (dtype, rows, cols, pitch)
    if rows * cols >= 64 * 64 and pitch == cols + 3:
        fma_step, _ = _run_plan(u, coeffs, T, dtype=npd, cols=cols, path=dtb.PATH_STEP)
        fma_dtb, d = _run_plan(u, coeffs, T, dtype=npd, cols=cols, path=dtb.PATH_RESIDENT, ghost_k=3)
        assert d["path"] == dtb.PATH_RESIDENT
        assert np.array_equal(fma_step, fma_dtb)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_box_fma_default_within_tolerance(dtype):
    rows, cols, T = 700, 900, 120
    rng = np.random.default_rng(5)
    coeffs = inputs.box_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols)
    npd = np.float64 if dtype == "f64" else np.float32
    _say("box fma", dtype, rows, cols, T)
    got, desc = _run_plan(u.astype(npd), coeffs, T, dtype=npd)
    assert desc["exact"] == 0 and desc["stencil"] == 9
    ref = oracle.j2d9pt_f64(u.astype(npd).astype(np.float64), np.array(coeffs, dtype=npd).astype(np.float64), T)
    err = oracle.rel_max_err(got, ref)
    assert err <= (TOL_F64 if dtype == "f64" else f32_bound9(T)), err


def test_box_fma_tiling_invariant():
    """The fused chain per cell does not depend on how the grid is tiled: resident at two exchange depths and
    the sweep agree bit for bit."""
    rows, cols, T = 640, 900, 45
    coeffs = inputs.box_weights(78)
    u = inputs.uniform_grid(rows, cols, 79, halo=0.25)
    _say("box tiling invariance", rows, cols, T)
    a, _ = _run_plan(u, coeffs, T, path=dtb.PATH_RESIDENT, ghost_k=3)
    b, _ = _run_plan(u, coeffs, T, path=dtb.PATH_RESIDENT, ghost_k=11)
    c, d = _run_plan(u, coeffs, T, path=dtb.PATH_SWEEP, ghost_k=4, depth_D=20, max_wg=12)
    assert d["path"] == dtb.PATH_SWEEP
    assert np.array_equal(a, b) and np.array_equal(a, c)


@pytest.mark.parametrize("path,extra", [(dtb.PATH_RESIDENT, dict(ghost_k=5)),
                                        (dtb.PATH_SWEEP, dict(ghost_k=4, depth_D=13, max_wg=9))],
                         ids=["resident", "sweep"])
def test_box_nan_poison_never_reaches_results(path, extra):
    """Cells outside every tile's fresh ring and the exchange buffers are NaN-filled at each exchange; the
    box reads the diagonal ghost cells too, so a missing corner of the ring would show."""
    rows, cols, T = 420, 650, 47
    rng = np.random.default_rng(191)
    coeffs = inputs.box_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols)
    _say("box poison", path, rows, cols, T)
    got, _ = _run_plan(u, coeffs, T, path=path, exact=True, debug=dtb.DEBUG_POISON, **extra)
    assert not np.isnan(got).any()
    assert np.array_equal(got, oracle.j2d9pt_f64(u, coeffs, T))


@pytest.mark.parametrize("case", [((300, 260), dict(path=dtb.PATH_RESIDENT, ghost_k=1)),
                                  ((300, 260), dict(path=dtb.PATH_RESIDENT, ghost_k=7)),
                                  ((517, 389), dict(path=dtb.PATH_RESIDENT, ghost_k=14)),
                                  ((700, 650), dict(path=dtb.PATH_SWEEP, ghost_k=6, depth_D=16, max_wg=6))],
                         ids=lambda c: f"{c[0][0]}x{c[0][1]}-k{c[1]['ghost_k']}")
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_box_staged_and_direct_exchange_agree(dtype, case):
    (rows, cols), opts = case
    npd = np.float64 if dtype == "f64" else np.float32
    ref_fn = oracle.j2d9pt_f64 if dtype == "f64" else oracle.j2d9pt_f32
    rng = np.random.default_rng(141 + rows + cols)
    coeffs = inputs.box_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols).astype(npd)
    T = 3 * opts["ghost_k"] + 2
    ref = ref_fn(u, coeffs, T)
    for debug in (0, dtb.DEBUG_DIRECT_XCHG):
        _say("box staged/direct", dtype, rows, cols, opts, "debug", debug, "T", T)
        got, _ = _run_plan(u, coeffs, T, dtype=npd, exact=True, debug=debug, **opts)
        assert np.array_equal(got, ref), (rows, cols, opts, debug)


def test_box_tuned_plan_is_correct():
    rows, cols, T = 500, 600, 30
    coeffs = inputs.box_weights(3)
    u = inputs.uniform_grid(rows, cols, 4, halo=0.5)
    _say("box tuned", rows, cols, T)
    got, desc = _run_plan(u, coeffs, T, tune=True, exact=True)
    assert desc["stencil"] == 9
    assert np.array_equal(got, oracle.j2d9pt_f64(u, coeffs, T))


def test_box_halo_padding_untouched_and_five_coefficients_refused():
    rows, cols, pitch = 100, 130, 140
    u = inputs.uniform_grid(rows, cols, 8, halo=0.7, pitch=pitch)
    u[:, cols + 2:] = -5.0
    coeffs = inputs.box_weights(8)
    _say("box padding", rows, cols, pitch)
    got, _ = _run_plan(u, coeffs, 9, cols=cols, exact=True)
    assert np.array_equal(got[0], u[0]) and np.array_equal(got[-1], u[-1])
    assert np.array_equal(got[:, 0], u[:, 0]) and np.array_equal(got[:, cols + 1:], u[:, cols + 1:])
    assert np.array_equal(got, oracle.j2d9pt_f64(u, coeffs, 9, cols=cols))
    g = _dev(u)
    plan = dtb.plan_for(g, 9, cols=cols, stencil=9)
    with pytest.raises(ValueError):
        plan.run(g, inputs.EQUAL_WEIGHTS, 9, cols=cols)
    plan.destroy()


@pytest.mark.slow
@pytest.mark.parametrize("name", ["j2d9pt_2048x2048_f64_T10000", "j2d9pt_8192x8192_f64_T1000",
                                  "j2d9pt_8192x8192_f32_T1000"])
def test_box_full_size_default_plan(name, capsys):
    """The benchmark's box workloads in the launch configuration it times (the default plan), whole grid, all
    steps, against the oracle (FP64 tolerance; FP32 against the FP64 oracle within its bound)."""
    w = inputs.workload(name)
    u0 = w.grid()
    npd = np.float64 if w.dtype == "f64" else np.float32
    with capsys.disabled():
        _say("box full size", w.name)
        g = _dev(u0.astype(npd))
        plan = dtb.plan_for(g, w.T, stencil=9)
        desc = plan.describe()
        plan.run(g, w.coeffs, w.T)
        plan.check()
        got = g.cpu().numpy()
        del g
        plan.destroy()
        ref = oracle_in_chunks(oracle.j2d9pt_f64, u0.astype(npd).astype(np.float64),
                               np.array(w.coeffs, dtype=npd).astype(np.float64), w.T, w.name)
    err = oracle.rel_max_err(got, ref)
    tol = TOL_F64 if w.dtype == "f64" else f32_bound9(w.T)
    record(workload=w.name, dtype=w.dtype, plan=desc, rel_max_err_vs_fp64_oracle=err, tolerance=tol)
    assert desc["stencil"] == 9
    # The box's register tiles are smaller than j2d5pt's (FP64 64 x 256): even 2048^2 does not fit on chip at
    # once and is swept, in two big tiles.
    assert desc["path"] == dtb.PATH_SWEEP, desc
    assert err <= tol, err
