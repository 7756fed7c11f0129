"""GPU parity: libdtb (through its C ABI) against the CPU oracle.

Exact mode (separately rounded products summed W, E, S, C, N) must match the
oracle bit for bit -- FP64 against the FP64 oracle, FP32 against the FP32
oracle.  The default fused chain must stay within 1e-13 relative max-norm of
the FP64 oracle.  Every case prints its parameters before it touches the GPU.
"""
import math
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


def f32_bound(T):
    """A priori relative max-norm bound of the FP32 path against the FP64 oracle for non-negative
    weights summing to 1 (each step is a convex combination, so errors do not grow): at most five
    roundings per cell per step, one rounding of each input cell and of each weight (the latter
    acting once per step), doubled for safety: 2 (6T + 1) u."""
    return 2 * (6 * T + 1) * U_F32


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _dev(u):
    return torch.from_numpy(np.ascontiguousarray(u)).to("cuda")


def _random_halo(u, rng, rows, cols):
    u[0, :cols + 2] = rng.uniform(-1, 2, cols + 2)
    u[rows + 1, :cols + 2] = rng.uniform(-1, 2, cols + 2)
    u[:, 0] = rng.uniform(-1, 2, rows + 2)
    u[:, cols + 1] = rng.uniform(-1, 2, rows + 2)
    return u


def _run_plan(u, coeffs, T, dtype=np.float64, cols=None, **opts):
    g = _dev(u.astype(dtype))
    plan = dtb.plan_for(g, T, cols=cols, **opts)
    plan.run(g, coeffs, T, cols=cols)
    plan.check()
    desc = plan.describe()
    out = g.cpu().numpy()
    plan.destroy()
    return out, desc


SHAPES = [(1, 1), (1, 37), (45, 1), (3, 200), (127, 131), (256, 256), (200, 300), (70, 130), (129, 257)]


# FP64 register tiles (rows x columns) by rows per lane: 2 columns per lane, or 4 at R = 12.
F64_TILE = {8: (64, 128), 12: (96, 256), 16: (128, 128), 24: (192, 128)}


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("R", [8, 12, 16, 24])
def test_exact_f64_bitwise(shape, R):
    rows, cols = shape
    rng = np.random.default_rng(rows * 1000 + cols + R)
    coeffs = inputs.dirichlet_weights(rng)
    u_var = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols)  # halo changes along each side
    u_const = inputs.uniform_grid(rows, cols, rng, halo=0.625)                   # constant nonzero halo
    for i, ((k, T), u) in enumerate(zip([(1, 3), (2, 7), (4, 4), (5, 23), (8, 37), (16, 9), (3, 17), (8, 40)],
                                        [u_var, u_var, u_var, u_var, u_var, u_var, u_const, u_const])):
        _say("exact f64", rows, cols, "R", R, "k", k, "T", T)
        try:
            got, desc = _run_plan(u, coeffs, T, path=dtb.PATH_RESIDENT, ghost_k=k, rows_per_lane=R, exact=True)
        except dtb.DtbError as e:
            # Only the largest tiles may be unavailable: their exact variants for grids narrower than
            # the tile spill registers, and the planner never picks a spilling kernel.  The refusal
            # depends on the shape and R only, so it comes at the first case or not at all.
            er, ec = F64_TILE[R]
            assert i == 0 and e.status == -3 and R in (12, 24) and (rows < er or cols < ec), (rows, cols, R, k, e)
            pytest.skip(f"exact FP64 kernel with {R} rows per lane for a {rows}x{cols} grid (narrower than its "
                        f"{er}x{ec} tile) spills registers; the planner refuses it (DTB_ERR_NOT_CORESIDENT)")
        ref = oracle.j2d5pt_f64(u, coeffs, T)
        assert desc["path"] == dtb.PATH_RESIDENT and desc["exact"] == 1
        assert np.array_equal(got, ref), (rows, cols, R, k, T, float(np.max(np.abs(got - ref))))


@pytest.mark.parametrize("shape", [(1, 1), (40, 1), (2, 300), (131, 127), (256, 256), (90, 520), (517, 389)],
                         ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("R", [8, 16, 24])
def test_exact_f32_bitwise(shape, R):
    rows, cols = shape
    rng = np.random.default_rng(rows * 7 + cols + R)
    coeffs = (0.05, 0.4, 0.01, 0.5, 0.04)  # strongly asymmetric: drives cells into subnormals
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols).astype(np.float32)
    for i, (k, T) in enumerate([(2, 5), (6, 40), (8, 200), (11, 60), (12, 50)]):
        _say("exact f32", rows, cols, "R", R, "k", k, "T", T)
        try:
            got, _ = _run_plan(u, coeffs, T, dtype=np.float32, path=dtb.PATH_RESIDENT, ghost_k=k,
                               rows_per_lane=R, exact=True)
        except dtb.DtbError as e:
            # The resident exact FP32 kernels with 24 rows per lane spill registers when the grid is
            # narrower than their 192 x 256 tile (the row/column-checking variants); the planner never
            # picks a spilling kernel.  The full-size variant does not spill and runs below.
            assert i == 0 and e.status == -3 and R == 24 and (rows < 192 or cols < 256), (rows, cols, R, k, e)
            pytest.skip(f"exact FP32 kernel with 24 rows per lane for a {rows}x{cols} grid (narrower than its "
                        "192x256 tile) spills registers; the planner refuses it (DTB_ERR_NOT_CORESIDENT)")
        ref = oracle.j2d5pt_f32(u, coeffs, T)
        assert np.array_equal(got, ref), (rows, cols, R, k, T)


@pytest.mark.parametrize("shape", [(517, 389), (700, 900), (1000, 1300)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_f32_r24_production_tile(shape):
    """The FP32 tile the planner picks for 3072^2 (resident) and 16384^2 (swept): 24 rows x 4 columns per
    lane at exchange depths 11 and 12.  Exact mode must equal the FP32 oracle bit for bit, resident and
    swept; the default fused chain must equal the same chain computed with 8-row tiles bit for bit (the
    chain per cell does not depend on the tiling), resident and swept."""
    rows, cols = shape
    rng = np.random.default_rng(rows + cols)
    coeffs = inputs.dirichlet_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols).astype(np.float32)
    T = 61
    ref32 = oracle.j2d5pt_f32(u, coeffs, T)
    fma8, d8 = _run_plan(u, coeffs, T, dtype=np.float32, path=dtb.PATH_RESIDENT, ghost_k=4, rows_per_lane=8)
    assert d8["rows_per_lane"] == 8 and d8["exact"] == 0
    for k in (11, 12):
        for path, extra in ((dtb.PATH_RESIDENT, {}), (dtb.PATH_SWEEP, dict(depth_D=3 * k, max_wg=6))):
            _say("f32 R24", rows, cols, "k", k, "path", path, "T", T)
            got, desc = _run_plan(u, coeffs, T, dtype=np.float32, path=path, ghost_k=k, rows_per_lane=24,
                                  exact=True, **extra)
            assert desc["rows_per_lane"] == 24 and desc["cols_per_lane"] == 4 and desc["exact"] == 1, desc
            assert desc["path"] == path and (path == dtb.PATH_RESIDENT or desc["big_tiles"] >= 2), desc
            assert np.array_equal(got, ref32), ("exact", rows, cols, k, path)
            fma, desc = _run_plan(u, coeffs, T, dtype=np.float32, path=path, ghost_k=k, rows_per_lane=24, **extra)
            assert desc["rows_per_lane"] == 24 and desc["exact"] == 0, desc
            assert np.array_equal(fma, fma8), ("fma", rows, cols, k, path)


def test_exact_f32_keeps_subnormals():
    rows, cols = 64, 300
    coeffs = (0.05, 0.4, 0.01, 0.5, 0.04)
    u = inputs.uniform_grid(rows, cols, 3).astype(np.float32)
    T = 400
    _say("f32 subnormals", rows, cols, T)
    got, _ = _run_plan(u, coeffs, T, dtype=np.float32, path=dtb.PATH_RESIDENT, exact=True)
    ref = oracle.j2d5pt_f32(u, coeffs, T)
    tiny = np.finfo(np.float32).tiny
    sub = (ref[1:-1, 1:-1] != 0) & (np.abs(ref[1:-1, 1:-1]) < tiny)
    assert sub.any(), "the case should produce subnormal values"
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("shape", [(1, 1), (127, 131), (300, 700)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_step_path_bitwise_and_matches_dtb_fma(shape):
    rows, cols = shape
    rng = np.random.default_rng(5)
    coeffs = inputs.dirichlet_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols)
    for T in (1, 2, 9):
        _say("step path", rows, cols, "T", T)
        got, desc = _run_plan(u, coeffs, T, path=dtb.PATH_STEP, exact=True)
        assert desc["path"] == dtb.PATH_STEP
        assert np.array_equal(got, oracle.j2d5pt_f64(u, coeffs, T))
        step_fma, _ = _run_plan(u, coeffs, T, path=dtb.PATH_STEP)
        dtb_fma, _ = _run_plan(u, coeffs, T, path=dtb.PATH_RESIDENT, ghost_k=4)
        # The fused chains agree bit for bit except where DTB folds the west/east
        # halo product into the chain's addend (first and last interior column),
        # which changes one rounding there; the difference spreads one column per step.
        if cols > 2 * T + 2:
            assert np.array_equal(step_fma[:, T + 1:cols - T], dtb_fma[:, T + 1:cols - T])
        assert oracle.rel_max_err(dtb_fma, step_fma) < 1e-15


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape_pitch", [(1, 1, 4), (64, 1, 4), (33, 130, 132), (129, 254, 256), (129, 255, 260),
                                         (200, 510, 513), (77, 2046, 2048)],
                         ids=lambda s: f"{s[0]}x{s[1]}p{s[2]}")
def test_step_kernel_both_access_widths_bitwise(dtype, shape_pitch):
    """The one-step baseline uses one 16-byte access per lane when rows start 16-byte aligned (pitch a
    multiple of 2 FP64 / 4 FP32 values) and one 8- or 4-byte access otherwise; exact mode equals the oracle
    bit for bit either way, pitch padding untouched."""
    rows, cols, pitch = shape_pitch
    npd = np.float64 if dtype == "f64" else np.float32
    rng = np.random.default_rng(rows + cols + pitch)
    coeffs = inputs.dirichlet_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng, pitch=pitch), rng, rows, cols).astype(npd)
    u[:, cols + 2:] = -9.0
    ref_fn = oracle.j2d5pt_f64 if dtype == "f64" else oracle.j2d5pt_f32
    for T in (1, 2, 5):
        _say("step kernel", dtype, rows, cols, pitch, "T", T)
        got, desc = _run_plan(u, coeffs, T, dtype=npd, cols=cols, path=dtb.PATH_STEP, exact=True)
        assert np.array_equal(got, ref_fn(u, coeffs, T, cols=cols)), (rows, cols, pitch, T)
        assert np.array_equal(got[:, cols + 2:], u[:, cols + 2:])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fma_default_within_tolerance(dtype):
    rows, cols, T = 600, 700, 300
    coeffs = inputs.dirichlet_weights(17)
    u = inputs.uniform_grid(rows, cols, 18, halo=0.5)
    _say("fma default", dtype, rows, cols, T)
    npd = np.float64 if dtype == "f64" else np.float32
    got, desc = _run_plan(u.astype(npd), coeffs, T, dtype=npd)
    assert desc["exact"] == 0
    assert got.dtype == npd
    ref = oracle.j2d5pt_f64(u, coeffs, T)
    err = oracle.rel_max_err(got, ref)
    print(f"[result] {dtype} fused chain rel max err vs FP64 oracle: {err:.3e}")
    if dtype == "f64":
        assert err <= TOL_F64
    else:
        assert 1e-9 < err <= f32_bound(T)  # an FP32 result cannot be closer than a few FP32 roundings


def test_halo_and_pitch_padding_untouched():
    rows, cols, pitch = 150, 140, 150
    u = inputs.uniform_grid(rows, cols, 4, halo=0.25, pitch=pitch)
    u[:, cols + 2:] = -777.0
    _say("padding", rows, cols, pitch)
    got, _ = _run_plan(u, inputs.EQUAL_WEIGHTS, 11, cols=cols, path=dtb.PATH_RESIDENT, ghost_k=3, exact=True)
    assert np.array_equal(got[:, cols + 2:], u[:, cols + 2:])
    assert np.array_equal(got[0], u[0]) and np.array_equal(got[-1], u[-1])
    assert np.array_equal(got[:, 0], u[:, 0]) and np.array_equal(got[:, cols + 1], u[:, cols + 1])
    ref = oracle.j2d5pt_f64(u, inputs.EQUAL_WEIGHTS, 11, cols=cols)
    assert np.array_equal(got, ref)


def test_semigroup_and_determinism():
    rows, cols = 333, 444
    coeffs = inputs.dirichlet_weights(21)
    u = inputs.uniform_grid(rows, cols, 22)
    _say("semigroup", rows, cols)
    g = _dev(u)
    plan = dtb.plan_for(g, 0, ghost_k=6)
    plan.run(g, coeffs, 25)
    plan.run(g, coeffs, 40)
    plan.check()
    split = g.cpu().numpy()
    g2 = _dev(u)
    plan.run(g2, coeffs, 65)
    plan.check()
    assert np.array_equal(split, g2.cpu().numpy())
    g3 = _dev(u)
    plan.run(g3, coeffs, 65)
    plan.check()
    assert np.array_equal(g3.cpu().numpy(), g2.cpu().numpy())
    # a different tiling (k, rows per lane) gives the same bits: the chain per cell is fixed
    other, _ = _run_plan(u, coeffs, 65, ghost_k=2, rows_per_lane=8)
    assert np.array_equal(other, split)


def test_T0_and_cached_run():
    rows, cols = 100, 90
    u = inputs.uniform_grid(rows, cols, 23)
    g = _dev(u)
    _say("cached run", rows, cols)
    dtb.run(g, inputs.EQUAL_WEIGHTS, 0)
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), u)
    dtb.run(g, inputs.EQUAL_WEIGHTS, 13)
    dtb.run(g, inputs.EQUAL_WEIGHTS, 13)
    torch.cuda.synchronize()
    ref = oracle.j2d5pt_f64(u, inputs.EQUAL_WEIGHTS, 26)
    assert oracle.rel_max_err(g.cpu().numpy(), ref) <= TOL_F64


def test_batched_matches_single_runs():
    rng = np.random.default_rng(31)
    probs, refs = [], []
    for i, side in enumerate([130, 257, 64, 400]):
        coeffs = inputs.dirichlet_weights(rng)
        u = inputs.uniform_grid(side, side, rng)
        T = int(rng.integers(5, 60))
        dt = np.float64 if i % 2 == 0 else np.float32
        probs.append((_dev(u.astype(dt)), coeffs, T))
        refs.append(oracle.j2d5pt_f64(u.astype(dt).astype(np.float64), np.array(coeffs, dtype=dt).astype(np.float64), T))
    _say("batched", len(probs))
    dtb.run_batched(probs)
    torch.cuda.synchronize()
    for (g, coeffs, T), ref in zip(probs, refs):
        err = oracle.rel_max_err(g.cpu().numpy(), ref)
        assert err <= (TOL_F64 if g.dtype == torch.float64 else 2e-5), err


@pytest.mark.slow
def test_full_size_2048_T10000_against_oracle():
    """The benchmark's workload and launch configuration, whole grid, all 10000 steps."""
    w = inputs.workload("j2d5pt_2048x2048_f64_T10000")
    u0 = w.grid()
    _say("full size", w.name)
    g = _dev(u0)
    plan = dtb.plan_for(g, w.T)
    plan.run(g, w.coeffs, w.T)
    plan.check()
    got = g.cpu().numpy()
    desc = plan.describe()
    ref = oracle.j2d5pt_f64(u0, w.coeffs, w.T)
    err = oracle.rel_max_err(got, ref)
    record(workload=w.name, dtype="f64", plan=desc, rel_max_err_vs_fp64_oracle=err, tolerance=TOL_F64)
    assert desc["path"] == dtb.PATH_RESIDENT
    assert err <= TOL_F64
    assert np.array_equal(got[0], u0[0]) and np.array_equal(got[:, 0], u0[:, 0])


@pytest.mark.slow
def test_full_size_2048_three_synchronisation_designs_agree():
    """2048^2 FP64, 10000 steps, in the three designs the benchmark compares: neighbour-flag exchange (the
    default), a device-wide barrier at every exchange (Section 3.2 as printed) and overlapped per-workgroup
    blocking with no synchronisation (Section 2).  The fused chain per cell does not depend on the tiling,
    so all three give the same bits; the default is within 1e-13 of the oracle (checked above)."""
    w = inputs.workload("j2d5pt_2048x2048_f64_T10000")
    u0 = w.grid()
    outs = {}
    for label, opts in (("flags", {}), ("grid_barrier", dict(path=dtb.PATH_RESIDENT, sync=dtb.SYNC_GRID_BARRIER)),
                        ("overlapped", dict(path=dtb.PATH_OVERLAPPED))):
        _say("full size", w.name, label)
        g = _dev(u0)
        plan = dtb.plan_for(g, w.T, **opts)
        plan.run(g, w.coeffs, w.T)
        plan.check()
        outs[label] = (g.cpu().numpy(), plan.describe())
        plan.destroy()
        del g
    assert outs["grid_barrier"][1]["sync"] == 1 and outs["overlapped"][1]["path"] == dtb.PATH_OVERLAPPED
    for label in ("grid_barrier", "overlapped"):
        assert np.array_equal(outs[label][0], outs["flags"][0]), label
    record(workload=w.name, dtype="f64", design="overlapped", plan=outs["overlapped"][1],
           bitwise_equal_to_default_plan=True)


def test_sine_mode_full_size_closed_form():
    """2048^2, 10000 steps of a single sine mode against its closed-form decay (symmetrised weights)."""
    rows = cols = 2048
    c, n, s, e, w = inputs.workload("j2d5pt_2048x2048_f64_T10000").coeffs
    for coeffs in [(c, (n + s) / 2, (n + s) / 2, (e + w) / 2, (e + w) / 2), inputs.EQUAL_WEIGHTS]:
        u0 = inputs.sine_grid(rows, cols)
        T = 10000
        _say("sine mode", coeffs)
        g = _dev(u0)
        plan = dtb.plan_for(g, T)
        plan.run(g, coeffs, T)
        plan.check()
        got = g.cpu().numpy()
        cc, nn, ss, ee, ww = coeffs
        lam = cc + 2 * math.sqrt(nn * ss) * math.cos(math.pi / (rows + 1)) + 2 * math.sqrt(ee * ww) * math.cos(
            math.pi / (cols + 1))
        want = u0 * math.exp(T * math.log(lam))
        err = np.max(np.abs(got[1:-1, 1:-1] - want[1:-1, 1:-1])) / np.max(np.abs(want[1:-1, 1:-1]))
        print(f"[result] sine mode lambda^T={lam ** T:.6f} rel err {err:.3e}")
        assert err < 1e-11


# ----------------------------------------------------------------------------- tile-serial sweep

@pytest.mark.parametrize("case", [
    # rows, cols, max_wg, k, D, T, R
    (600, 700, 8, 4, 16, 37, 8),      # several big tiles, T not a multiple of D, odd rounds
    (600, 700, 8, 3, 10, 40, 8),      # even rounds
    (1000, 333, 6, 5, 12, 25, 16),
    (300, 1100, 12, 6, 20, 61, 8),
    (257, 129, 4, 2, 7, 9, 8),
    (130, 900, 8, 4, 9, 5, 8),        # T < D: one short round
], ids=lambda c: "x".join(map(str, c)))
def test_sweep_exact_bitwise(case):
    rows, cols, max_wg, k, D, T, R = case
    rng = np.random.default_rng(rows + 7 * cols + T)
    coeffs = inputs.dirichlet_weights(rng)
    u_var = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols)
    u_const = inputs.uniform_grid(rows, cols, rng, halo=0.375)
    for u in (u_var, u_const):
        _say("sweep f64", case)
        got, desc = _run_plan(u, coeffs, T, path=dtb.PATH_SWEEP, ghost_k=k, depth_D=D, max_wg=max_wg,
                              rows_per_lane=R, exact=True)
        assert desc["path"] == dtb.PATH_SWEEP and desc["depth_D"] == D and desc["big_tiles"] >= 2, desc
        ref = oracle.j2d5pt_f64(u, coeffs, T)
        assert np.array_equal(got, ref), (case, float(np.max(np.abs(got - ref))))


def test_sweep_plan_reused_across_runs():
    """A sweep plan whose big tiles leave some workgroups idle, run several times in a row: every
    run must start from consistent epoch flags (regression: idle workgroups once ended a run behind)."""
    rows, cols = 900, 500
    coeffs = inputs.dirichlet_weights(95)
    u = inputs.uniform_grid(rows, cols, 96)
    g = _dev(u)
    plan = dtb.plan_for(g, 0, path=dtb.PATH_SWEEP, ghost_k=4, depth_D=12, max_wg=10, rows_per_lane=8, exact=True)
    assert plan.describe()["big_tiles"] >= 3
    total = 0
    for T in (7, 30, 13, 25):
        _say("sweep reuse", T)
        plan.run(g, coeffs, T)
        plan.check()
        total += T
    assert np.array_equal(g.cpu().numpy(), oracle.j2d5pt_f64(u, coeffs, total))
    plan.destroy()


def test_sweep_exact_f32_bitwise():
    rows, cols, T = 500, 1300, 33
    rng = np.random.default_rng(77)
    coeffs = inputs.dirichlet_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols).astype(np.float32)
    _say("sweep f32", rows, cols, T)
    got, desc = _run_plan(u, coeffs, T, dtype=np.float32, path=dtb.PATH_SWEEP, ghost_k=4, depth_D=14, max_wg=10,
                          rows_per_lane=8, exact=True)
    assert desc["big_tiles"] >= 2
    assert np.array_equal(got, oracle.j2d5pt_f32(u, coeffs, T))


def test_sweep_fma_matches_resident_fma():
    """Same fused chain per cell whichever way the grid is tiled."""
    rows, cols, T = 700, 900, 45
    coeffs = inputs.dirichlet_weights(78)
    u = inputs.uniform_grid(rows, cols, 79, halo=0.25)
    _say("sweep vs resident", rows, cols, T)
    sw, d1 = _run_plan(u, coeffs, T, path=dtb.PATH_SWEEP, ghost_k=4, depth_D=20, max_wg=12, rows_per_lane=8)
    rs, d2 = _run_plan(u, coeffs, T, path=dtb.PATH_RESIDENT, ghost_k=4, rows_per_lane=8)
    assert d1["path"] == dtb.PATH_SWEEP and d2["path"] == dtb.PATH_RESIDENT
    assert np.array_equal(sw, rs)


@pytest.mark.slow
def test_sweep_full_size_8192_T1000():
    """8192^2 FP64, 1000 steps, halo 1.0: the default plan (tile-serial sweep) against the oracle."""
    w = inputs.workload("j2d5pt_8192x8192_f64_T1000")
    u0 = w.grid()
    _say("full size", w.name)
    g = _dev(u0)
    plan = dtb.plan_for(g, w.T)
    desc = plan.describe()
    assert desc["path"] == dtb.PATH_SWEEP, desc
    plan.run(g, w.coeffs, w.T)
    plan.check()
    got = g.cpu().numpy()
    del g
    ref = oracle.j2d5pt_f64(u0, w.coeffs, w.T)
    err = oracle.rel_max_err(got, ref)
    record(workload=w.name, dtype="f64", plan=desc, rel_max_err_vs_fp64_oracle=err, tolerance=TOL_F64)
    assert err <= TOL_F64


# ----------------------------------------------------------------------------- batched launch

def _batch_refs(probs):
    refs = []
    for g, coeffs, T in probs:
        u = g.cpu().numpy()
        dt = u.dtype
        refs.append(oracle.j2d5pt_f64(u.astype(np.float64), np.array(coeffs, dtype=dt).astype(np.float64), T))
    return refs


def test_batched_mixed_with_sweep_job_and_replay():
    rng = np.random.default_rng(41)
    shapes = [(130, 130, np.float64, 37), (257, 300, np.float32, 21), (64, 700, np.float32, 9), (1, 1, np.float64, 5),
              (400, 410, np.float64, 50), (2100, 2100, np.float64, 30), (90, 3000, np.float64, 12)]
    for call in range(2):  # the second call replays the graph with new grids and coefficients
        probs = []
        for rows, cols, dt, T in shapes:
            coeffs = inputs.dirichlet_weights(rng)
            u = inputs.uniform_grid(rows, cols, rng, halo=float(rng.uniform(0, 1)))
            probs.append((_dev(u.astype(dt)), coeffs, T))
        refs = _batch_refs(probs)
        _say("batched call", call)
        dtb.run_batched(probs)
        dtb.batch_check()
        for (g, coeffs, T), ref, shp in zip(probs, refs, shapes):
            err = oracle.rel_max_err(g.cpu().numpy(), ref)
            assert err <= (TOL_F64 if g.dtype == torch.float64 else 2e-5), (shp, err)


def test_batched_equals_single_runs_fma():
    """The batched kernel's fused chain per cell equals the single-grid kernels' (same tiling-invariant chain)."""
    rng = np.random.default_rng(43)
    shapes = [(200, 300, np.float64, 40), (333, 257, np.float32, 33), (150, 700, np.float64, 17)]
    probs, singles = [], []
    for rows, cols, dt, T in shapes:
        coeffs = inputs.dirichlet_weights(rng)
        u = inputs.uniform_grid(rows, cols, rng).astype(dt)
        probs.append((_dev(u), coeffs, T))
        s, _ = _run_plan(u, coeffs, T, dtype=dt, path=dtb.PATH_RESIDENT)
        singles.append(s)
    _say("batched vs single")
    dtb.run_batched(probs)
    dtb.batch_check()
    for (g, _, _), s in zip(probs, singles):
        assert np.array_equal(g.cpu().numpy(), s)


# ----------------------------------------------------------------------------- debug aids, tuner, failure path

@pytest.mark.parametrize("path,extra", [(dtb.PATH_RESIDENT, dict(ghost_k=5, rows_per_lane=8)),
                                        (dtb.PATH_SWEEP, dict(ghost_k=4, depth_D=13, max_wg=9, rows_per_lane=8))],
                         ids=["resident", "sweep"])
def test_nan_poison_never_reaches_results(path, extra):
    """Cells outside every tile's fresh ring and the exchange buffers are NaN-filled at each exchange;
    the results must still equal the oracle bit for bit."""
    rows, cols, T = 420, 650, 47
    rng = np.random.default_rng(91)
    coeffs = inputs.dirichlet_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols)
    _say("poison", path, rows, cols, T)
    got, _ = _run_plan(u, coeffs, T, path=path, exact=True, debug=dtb.DEBUG_POISON, **extra)
    assert not np.isnan(got).any()
    assert np.array_equal(got, oracle.j2d5pt_f64(u, coeffs, T))


def test_watchdog_reports_timeout_and_drains():
    """With the bounded waits cut to a few polls some workgroup gives up: the run still ends and
    dtb_plan_check reports DTB_ERR_TIMEOUT (or, if nobody had to wait, the result is right)."""
    rows, cols, T = 900, 900, 64
    u = inputs.uniform_grid(rows, cols, 92)
    g = _dev(u)
    plan = dtb.plan_for(g, T, path=dtb.PATH_RESIDENT, ghost_k=2, rows_per_lane=8, debug=dtb.DEBUG_TINY_SPIN)
    assert plan.describe()["workgroups"] > 8
    _say("watchdog")
    plan.run(g, inputs.EQUAL_WEIGHTS, T)
    try:
        plan.check()
        timed_out = False
    except dtb.DtbError as e:
        assert e.status == -6
        timed_out = True
    if not timed_out:
        assert oracle.rel_max_err(g.cpu().numpy(), oracle.j2d5pt_f64(u, inputs.EQUAL_WEIGHTS, T)) <= TOL_F64
    plan.destroy()
    # a normal plan afterwards works
    got, _ = _run_plan(u, inputs.EQUAL_WEIGHTS, 10, path=dtb.PATH_RESIDENT)
    assert oracle.rel_max_err(got, oracle.j2d5pt_f64(u, inputs.EQUAL_WEIGHTS, 10)) <= TOL_F64


def test_sweep_watchdog_reports_timeout_and_drains():
    """The tile-serial sweep's bounded waits (exchange flags, the split-phase barrier between big tiles, the
    device barrier at the end of a round) cut to a few polls: the run still ends, and dtb_plan_check reports
    DTB_ERR_TIMEOUT (or, if nobody had to wait, the result is right)."""
    rows, cols, T = 3000, 3000, 40
    u = inputs.uniform_grid(rows, cols, 94)
    g = _dev(u)
    plan = dtb.plan_for(g, T, path=dtb.PATH_SWEEP, ghost_k=4, depth_D=16, rows_per_lane=8,
                        debug=dtb.DEBUG_TINY_SPIN)
    d = plan.describe()
    assert d["path"] == dtb.PATH_SWEEP and d["big_tiles"] >= 2, d
    _say("sweep watchdog", d["big_tiles"], "big tiles")
    plan.run(g, inputs.EQUAL_WEIGHTS, T)
    try:
        plan.check()
        timed_out = False
    except dtb.DtbError as e:
        assert e.status == -6
        timed_out = True
    if not timed_out:
        assert oracle.rel_max_err(g.cpu().numpy(), oracle.j2d5pt_f64(u, inputs.EQUAL_WEIGHTS, T)) <= TOL_F64
    plan.destroy()
    # a normal sweep plan afterwards works
    got, _ = _run_plan(u, inputs.EQUAL_WEIGHTS, 20, path=dtb.PATH_SWEEP, ghost_k=4, depth_D=16, rows_per_lane=8)
    assert oracle.rel_max_err(got, oracle.j2d5pt_f64(u, inputs.EQUAL_WEIGHTS, 20)) <= TOL_F64


def test_tuned_plan_is_correct():
    rows, cols, T = 1500, 1700, 120
    coeffs = inputs.dirichlet_weights(93)
    u = inputs.uniform_grid(rows, cols, 94)
    _say("tuner", rows, cols)
    got, desc = _run_plan(u, coeffs, T, tune=True)
    print(f"[result] tuned plan {desc}")
    assert oracle.rel_max_err(got, oracle.j2d5pt_f64(u, coeffs, T)) <= TOL_F64


def test_phase_clocks_do_not_change_results():
    rows, cols, T, k = 500, 700, 60, 6
    coeffs = inputs.dirichlet_weights(31)
    u = inputs.uniform_grid(rows, cols, 32)
    _say("phase clocks", rows, cols, "T", T, "k", k)
    g = _dev(u)
    plan = dtb.plan_for(g, T, path=dtb.PATH_RESIDENT, ghost_k=k, exact=True, debug=dtb.DEBUG_TIMING)
    plan.run(g, coeffs, T)
    plan.check()
    clocks = plan.timing()
    assert np.array_equal(g.cpu().numpy(), oracle.j2d5pt_f64(u, coeffs, T))
    assert len(clocks) == plan.describe()["workgroups"]
    for c in clocks:
        assert c["exchanges"] == (T + k - 1) // k - 1
        parts = c["steps"] + c["publish"] + c["wait"] + c["ghost"] + c["stage_out"] + c["stage_in"]
        assert abs(c["total"] - parts) < 1e-6
    assert all(v == 0 for c in plan.timing() for v in c.values())  # reading resets them
    plan.destroy()


STAGED_DIRECT_CASES = [
    ((300, 260), dict(path=dtb.PATH_RESIDENT, ghost_k=1, rows_per_lane=8)),
    ((300, 260), dict(path=dtb.PATH_RESIDENT, ghost_k=7, rows_per_lane=8)),
    ((517, 389), dict(path=dtb.PATH_RESIDENT, ghost_k=12)),
    ((517, 389), dict(path=dtb.PATH_RESIDENT, ghost_k=16)),
    ((100, 3000), dict(path=dtb.PATH_RESIDENT, ghost_k=5, max_wg=40)),
    ((700, 650), dict(path=dtb.PATH_SWEEP, ghost_k=6, depth_D=16, max_wg=6)),
    ((450, 900), dict(path=dtb.PATH_RESIDENT, ghost_k=9, rows_per_lane=12)),
    ((450, 900), dict(path=dtb.PATH_RESIDENT, ghost_k=11, rows_per_lane=24, waves=4)),
]


def _case_id(c):
    (rows, cols), o = c
    return f"{rows}x{cols}-" + "-".join(f"{k}{v}" for k, v in o.items() if k != "path") + \
        ("-sweep" if o["path"] == dtb.PATH_SWEEP else "")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", STAGED_DIRECT_CASES, ids=_case_id)
def test_staged_and_direct_exchange_agree(dtype, case):
    # Border strips move through the LDS staging area unless the frames are too
    # large for it; the lane-by-lane path is forced with DEBUG_DIRECT_XCHG.  Both
    # must reproduce the oracle bit for bit, tiny tiles (frames without a hole)
    # and the resident / sweep paths included.
    (rows, cols), opts = case
    npd = np.float64 if dtype == "f64" else np.float32
    ref_fn = oracle.j2d5pt_f64 if dtype == "f64" else oracle.j2d5pt_f32
    if dtype == "f32" and (opts.get("waves") == 4 or opts.get("rows_per_lane") == 12):
        # Half-height workgroups exist for FP64 with 24 rows per lane only, and 12 rows per lane (the
        # 4-column FP64 tile) has no FP32 instance: both are refused before any HIP call.
        with pytest.raises(dtb.DtbError) as ei:
            dtb.Plan(rows, cols, cols + 2, dtb.F32, 0, exact=True, **opts)
        assert ei.value.status == -2
        return
    rng = np.random.default_rng(41 + rows + cols)
    coeffs = inputs.dirichlet_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols).astype(npd)
    T = 3 * opts["ghost_k"] + 2
    ref = ref_fn(u, coeffs, T)
    for debug in (0, dtb.DEBUG_DIRECT_XCHG):
        _say("staged/direct", dtype, rows, cols, opts, "debug", debug, "T", T)
        got, _ = _run_plan(u, coeffs, T, dtype=npd, exact=True, debug=debug, **opts)
        assert np.array_equal(got, ref), (rows, cols, opts, debug)


@pytest.mark.parametrize("shape", [(150, 300), (517, 389), (2048, 700)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_half_height_workgroups_bitwise(shape):
    # FP64, 24 rows per lane, 4 waves per workgroup (two workgroups per compute unit).
    rows, cols = shape
    rng = np.random.default_rng(rows + cols)
    coeffs = inputs.dirichlet_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols)
    for k, T in [(1, 3), (4, 21), (10, 45)]:
        _say("half-height", rows, cols, "k", k, "T", T)
        got, desc = _run_plan(u, coeffs, T, path=dtb.PATH_RESIDENT, ghost_k=k, rows_per_lane=24, waves=4,
                              exact=True)
        assert desc["waves"] == 4 and desc["ext_rows"] == 96
        assert np.array_equal(got, oracle.j2d5pt_f64(u, coeffs, T)), (rows, cols, k, T)


# ----------------------------------------------------------------------------- overlapped blocking, grid barrier

@pytest.mark.parametrize("shape", [(1, 1), (45, 1), (3, 200), (127, 131), (300, 700), (517, 389), (1000, 1300)],
                         ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("R", [8, 12, 24])
def test_overlapped_exact_f64_bitwise(shape, R):
    """Overlapped per-workgroup blocking (no inter-workgroup synchronisation, one launch per D steps): exact
    mode equals the oracle bit for bit for depths from 1 to 16, odd and even round counts, varying halo."""
    rows, cols = shape
    rng = np.random.default_rng(rows * 31 + cols + R)
    coeffs = inputs.dirichlet_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols)
    for i, (D, T) in enumerate([(1, 3), (2, 7), (5, 23), (8, 16), (16, 37)]):
        _say("overlapped f64", rows, cols, "R", R, "D", D, "T", T)
        try:
            got, desc = _run_plan(u, coeffs, T, path=dtb.PATH_OVERLAPPED, depth_D=D, rows_per_lane=R, exact=True)
        except dtb.DtbError as e:
            # As for the resident kernels: exact variants narrower than their tile spill for the largest
            # tiles, and are never chosen.
            er, ec = F64_TILE[R]
            assert i == 0 and e.status == -2 and R in (12, 24) and (rows < er or cols < ec), (rows, cols, R, e)
            pytest.skip(f"exact FP64 overlapped kernel with {R} rows per lane for a {rows}x{cols} grid (narrower "
                        f"than its {er}x{ec} tile) spills registers; the planner refuses it")
        assert desc["path"] == dtb.PATH_OVERLAPPED and desc["depth_D"] == D and desc["rows_per_lane"] == R
        assert np.array_equal(got, oracle.j2d5pt_f64(u, coeffs, T)), (rows, cols, R, D, T)


@pytest.mark.parametrize("R", [8, 24])
def test_overlapped_f32_exact_and_fma_tiling_invariant(R):
    rows, cols, T = 700, 1100, 45
    rng = np.random.default_rng(R)
    coeffs = inputs.dirichlet_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols).astype(np.float32)
    _say("overlapped f32", R)
    got, _ = _run_plan(u, coeffs, T, dtype=np.float32, path=dtb.PATH_OVERLAPPED, depth_D=6, rows_per_lane=R,
                       exact=True)
    assert np.array_equal(got, oracle.j2d5pt_f32(u, coeffs, T))
    fma, _ = _run_plan(u, coeffs, T, dtype=np.float32, path=dtb.PATH_OVERLAPPED, depth_D=7, rows_per_lane=R)
    res, _ = _run_plan(u, coeffs, T, dtype=np.float32, path=dtb.PATH_RESIDENT, ghost_k=4, rows_per_lane=8)
    assert np.array_equal(fma, res)


@pytest.mark.parametrize("shape", [(1, 1), (127, 131), (600, 700), (1000, 1300)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_grid_barrier_sync_exact_bitwise(shape):
    """The resident path with a device-wide barrier at every exchange point instead of neighbour flags."""
    rows, cols = shape
    rng = np.random.default_rng(rows + 3 * cols)
    coeffs = inputs.dirichlet_weights(rng)
    u = _random_halo(inputs.uniform_grid(rows, cols, rng), rng, rows, cols)
    for k, T in [(1, 4), (3, 17), (8, 40), (11, 45)]:
        _say("grid barrier", rows, cols, "k", k, "T", T)
        got, desc = _run_plan(u, coeffs, T, path=dtb.PATH_RESIDENT, ghost_k=k, sync=dtb.SYNC_GRID_BARRIER,
                              exact=True)
        assert desc["sync"] == 1
        assert np.array_equal(got, oracle.j2d5pt_f64(u, coeffs, T)), (rows, cols, k, T)
    # The same plan run twice in a row (the barrier counters are reset before every launch).
    g = _dev(u)
    plan = dtb.plan_for(g, 0, path=dtb.PATH_RESIDENT, ghost_k=5, sync=dtb.SYNC_GRID_BARRIER, exact=True)
    plan.run(g, coeffs, 12)
    plan.run(g, coeffs, 19)
    plan.check()
    assert np.array_equal(g.cpu().numpy(), oracle.j2d5pt_f64(u, coeffs, 31))
    plan.destroy()


def test_probes_measure_something():
    """The micro-benchmarks behind the measured roofline denominators run and report sane figures."""
    ms, byt = dtb.probe(dtb.PROBE_LDS_READ, iters=256)
    assert ms > 0 and byt > 0 and 1 < byt / (ms / 1e3) / 1e12 < 1000      # TB/s
    ms, byt = dtb.probe(dtb.PROBE_LDS_WRITE, iters=256)
    assert ms > 0 and 1 < byt / (ms / 1e3) / 1e12 < 1000
    ms, byt = dtb.probe(dtb.PROBE_COPY, size=64 << 20, iters=5)
    assert ms > 0 and 100 < byt / (ms / 1e3) / 1e9 < 100000                # GB/s
    ms, n = dtb.probe(dtb.PROBE_BARRIER, iters=100)
    assert n == 100 and 0.05 < ms * 1e3 / n < 1000                          # us per barrier
    ms, n = dtb.probe(dtb.PROBE_FLAGS, iters=100)
    assert n == 100 and 0.05 < ms * 1e3 / n < 1000
