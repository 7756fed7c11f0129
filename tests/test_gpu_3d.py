"""GPU parity of the 3-D seven-point stencil (j3d7pt): libdtb plans from dtb_plan3d, through the C ABI, against
the 3-D oracle (oracle/j3d7pt_oracle.c).

Exact mode (separately rounded products summed W, E, S, C, N, B, T) must match the oracle bit for bit, FP64
against the FP64 oracle and FP32 against the FP32 oracle, on the streaming path (1 to 3 steps per launch,
several z-blocks, tiles that meet the halo and tiles wider than the grid) and the one-step path.  The default
fused chain must stay within 1e-13 relative max-norm of the FP64 oracle and not depend on the tiling.  Every
case prints its parameters before it touches the GPU.
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


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _random_shell(u, rng):
    """A halo shell whose values change everywhere."""
    d, r, c = u.shape[0] - 2, u.shape[1] - 2, u.shape[2] - 2
    shell = np.ones(u.shape, dtype=bool)
    shell[1:d + 1, 1:r + 1, 1:c + 1] = False
    u[shell] = rng.uniform(-1, 2, int(shell.sum()))
    return u


def _err3(got, ref, cols):
    """The relative max-norm over the 3-D interior (the oracle's measure, applied to the interior cells laid
    out as one 2-D array inside a zero border it ignores)."""
    def flat(a):
        inner = np.asarray(a, dtype=np.float64)[1:-1, 1:-1, 1:cols + 1].reshape(-1, cols)
        return np.pad(inner, 1)
    return oracle.rel_max_err(flat(got), flat(ref))


def _run(u, coeffs, T, dtype=np.float64, cols=None, **opts):
    g = torch.from_numpy(np.ascontiguousarray(u.astype(dtype))).to("cuda")
    plan = dtb.plan3d_for(g, cols=cols, **opts)
    plan.run(g, coeffs, T, cols=cols)
    torch.cuda.synchronize()
    desc = plan.describe()
    out = g.cpu().numpy()
    plan.destroy()
    return out, desc


SHAPES = [(1, 1, 1), (3, 5, 7), (9, 40, 130), (17, 33, 300), (40, 70, 129), (5, 200, 90), (30, 64, 256)]


# (precision, columns per lane): every streaming instance.
INSTANCES = [("f64", 2), ("f32", 4), ("f32", 3)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("dtype,cpl", INSTANCES, ids=lambda v: str(v))
def test_3d_stream_exact_bitwise(shape, dtype, cpl):
    depth, rows, cols = shape
    npd = np.float64 if dtype == "f64" else np.float32
    ref_fn = oracle.j3d7pt_f64 if dtype == "f64" else oracle.j3d7pt_f32
    rng = np.random.default_rng(depth * 10007 + rows * 101 + cols)
    coeffs = inputs.weights7(rng)
    u = _random_shell(inputs.uniform_grid3(depth, rows, cols, rng), rng).astype(npd)
    for K, T, zb in [(3, 7, 0), (3, 3, 4), (2, 5, 3), (1, 4, 0), (3, 10, 5), (2, 1, 0)]:
        _say("3d exact", dtype, "cols/lane", cpl, shape, "K", K, "T", T, "zb", zb)
        got, desc = _run(u, coeffs, T, dtype=npd, path=dtb.PATH_STREAM3D, ghost_k=K, depth_D=zb, exact=True,
                         cols_per_lane=cpl)
        assert desc["path"] == dtb.PATH_STREAM3D and desc["stencil"] == 7 and desc["ghost_k"] == K, desc
        assert desc["cols_per_lane"] == cpl, desc
        ref = ref_fn(u, coeffs, T)
        assert np.array_equal(got, ref), (shape, K, T, zb, float(np.max(np.abs(got.astype(float) - ref))))


@pytest.mark.parametrize("shape", [(64, 40, 130), (50, 33, 300)], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("dtype,cpl", INSTANCES, ids=lambda v: str(v))
def test_3d_stream_exact_bitwise_deep_blocks(shape, dtype, cpl):
    """Deep z-blocks, so that most iterations of a workgroup run the streaming loop's branch-free steady state
    (every plane loaded ahead, every level producing an interior plane); shallow ones and the ends of the grid
    take the general form.  Both must equal the oracle bit for bit."""
    depth, rows, cols = shape
    npd = np.float64 if dtype == "f64" else np.float32
    ref_fn = oracle.j3d7pt_f64 if dtype == "f64" else oracle.j3d7pt_f32
    rng = np.random.default_rng(depth * 7 + rows * 3 + cols)
    coeffs = inputs.weights7(rng)
    u = _random_shell(inputs.uniform_grid3(depth, rows, cols, rng), rng).astype(npd)
    for K, T, zb in [(3, 7, depth), (3, 4, 30), (2, 5, 25), (1, 3, depth), (3, 9, 17)]:
        _say("3d exact deep", dtype, "cols/lane", cpl, shape, "K", K, "T", T, "zb", zb)
        got, desc = _run(u, coeffs, T, dtype=npd, path=dtb.PATH_STREAM3D, ghost_k=K, depth_D=zb, exact=True,
                         cols_per_lane=cpl)
        assert desc["path"] == dtb.PATH_STREAM3D and desc["ghost_k"] == K and desc["depth_D"] == zb, desc
        assert desc["cols_per_lane"] == cpl, desc
        ref = ref_fn(u, coeffs, T)
        assert np.array_equal(got, ref), (shape, K, T, zb, float(np.max(np.abs(got.astype(float) - ref))))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("shape_pitch", [(3, 4, 5, 8, 0), (9, 40, 130, 133, 42 * 133 + 5), (17, 33, 300, 302, 0)],
                         ids=lambda s: "x".join(map(str, s)))
def test_3d_step_path_bitwise_and_padding_untouched(dtype, shape_pitch):
    """The one-step baseline in exact mode equals the oracle bit for bit; pitch and plane padding stay
    untouched; the fused chain of the one-step kernel equals the streaming kernel's."""
    depth, rows, cols, pitch, pp = shape_pitch
    npd = np.float64 if dtype == "f64" else np.float32
    ref_fn = oracle.j3d7pt_f64 if dtype == "f64" else oracle.j3d7pt_f32
    rng = np.random.default_rng(depth + rows + cols + pitch)
    coeffs = inputs.weights7(rng)
    pp = pp or (rows + 2) * pitch
    # storage with plane padding: a (depth + 2) x pp buffer viewed as planes of (rows + 2) x pitch
    flat = np.full((depth + 2) * pp, -7.0)
    u = np.lib.stride_tricks.as_strided(flat, shape=(depth + 2, rows + 2, pitch), strides=(pp * 8, pitch * 8, 8))
    u[...] = _random_shell(inputs.uniform_grid3(depth, rows, cols, rng, pitch=pitch), rng)
    u[:, :, cols + 2:] = -5.0
    flat = flat.astype(npd)
    g = torch.from_numpy(flat).to("cuda").as_strided((depth + 2, rows + 2, pitch), (pp, pitch, 1))
    T = 5
    _say("3d step", dtype, shape_pitch)
    plan = dtb.plan3d_for(g, cols=cols, path=dtb.PATH_STEP, exact=True)
    plan.run(g, coeffs, T, cols=cols)
    torch.cuda.synchronize()
    got_flat = g.as_strided(((depth + 2) * pp,), (1,)).cpu().numpy()
    plan.destroy()
    dense = np.ascontiguousarray(np.lib.stride_tricks.as_strided(flat, shape=(depth + 2, rows + 2, pitch),
                                                                 strides=(pp * flat.itemsize, pitch * flat.itemsize,
                                                                          flat.itemsize)))
    ref = ref_fn(dense, coeffs, T, cols=cols)
    got = np.lib.stride_tricks.as_strided(got_flat, shape=(depth + 2, rows + 2, pitch),
                                          strides=(pp * flat.itemsize, pitch * flat.itemsize, flat.itemsize))
    assert np.array_equal(got, ref)
    # everything outside the planes' (rows + 2) x pitch boxes is plane padding
    mask = np.ones(got_flat.size, dtype=bool)
    for z in range(depth + 2):
        mask[z * pp:z * pp + (rows + 2) * pitch] = False
    assert np.all(got_flat[mask] == flat[mask])
    # fused chains agree between the one-step and the streaming kernels
    a, _ = _run(dense, coeffs, T, dtype=npd, cols=cols, path=dtb.PATH_STEP)
    b, _ = _run(dense, coeffs, T, dtype=npd, cols=cols, path=dtb.PATH_STREAM3D, ghost_k=3)
    assert np.array_equal(a, b)


def test_3d_fma_within_tolerance_and_tiling_invariant():
    depth, rows, cols, T = 40, 100, 300, 17
    rng = np.random.default_rng(5)
    coeffs = inputs.weights7(rng)
    u = _random_shell(inputs.uniform_grid3(depth, rows, cols, rng), rng)
    _say("3d fma", depth, rows, cols, T)
    a, d = _run(u, coeffs, T)
    assert d["exact"] == 0 and d["path"] == dtb.PATH_STREAM3D
    assert _err3(a, oracle.j3d7pt_f64(u, coeffs, T), cols) <= TOL_F64
    for K, zb in [(1, 0), (2, 7), (3, 3)]:
        b, _ = _run(u, coeffs, T, ghost_k=K, depth_D=zb)
        assert np.array_equal(a, b), (K, zb)


def test_3d_f32_instances_agree_bitwise_in_fused_mode():
    """The two FP32 streaming instances (4 and 3 columns per lane) compute each cell with the same fused chain
    in the same order, so the default mode gives the same bits whichever covers the grid; at 372 columns the
    planner takes 3 (two spans of 192 against two of 256)."""
    depth, rows, cols, T = 30, 64, 372, 11
    rng = np.random.default_rng(8)
    coeffs = inputs.weights7(rng)
    u = _random_shell(inputs.uniform_grid3(depth, rows, cols, rng), rng).astype(np.float32)
    _say("3d f32 instances", depth, rows, cols, T)
    a, d = _run(u, coeffs, T, dtype=np.float32)
    assert d["cols_per_lane"] == 3 and d["exact"] == 0, d
    for K, zb in [(3, 0), (2, 9), (1, 0)]:
        b, db = _run(u, coeffs, T, dtype=np.float32, ghost_k=K, depth_D=zb, cols_per_lane=4)
        assert db["cols_per_lane"] == 4, db
        assert np.array_equal(a, b), (K, zb)


def test_3d_plan_reuse_and_two_streams():
    """One plan, runs on two streams in a row: the second waits for the first (shared workspace)."""
    depth, rows, cols = 20, 50, 140
    coeffs = inputs.weights7(6)
    u = inputs.uniform_grid3(depth, rows, cols, 7, halo=0.25)
    g = torch.from_numpy(u).to("cuda")
    plan = dtb.plan3d_for(g, exact=True)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    _say("3d two streams")
    plan.run(g, coeffs, 4, stream=s1)
    plan.run(g, coeffs, 5, stream=s2)
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy(), oracle.j3d7pt_f64(u, coeffs, 9))
    plan.destroy()


def test_3d_rejects_2d_plans_and_five_coefficients():
    u = inputs.uniform_grid3(3, 4, 5, 1)
    g = torch.from_numpy(u).to("cuda")
    plan = dtb.plan3d_for(g)
    with pytest.raises(ValueError):
        plan.run(g, inputs.EQUAL_WEIGHTS, 1)
    g2 = torch.from_numpy(inputs.uniform_grid(4, 5, 1)).to("cuda")
    p2 = dtb.plan_for(g2)
    with pytest.raises(dtb.DtbError) as ei:
        dtb.Plan3D.run(p2, g, inputs.weights7(1), 1)
    assert ei.value.status == -8
    # a 3-D plan through the 2-D run call (the C ABI directly: the binding would refuse the coefficients)
    import ctypes
    grid2 = dtb._grid(g2)
    c5 = (ctypes.c_double * 5)(*inputs.EQUAL_WEIGHTS)
    assert dtb.load().dtb_run_plan(plan._h, ctypes.byref(grid2), c5, 1, dtb._stream(None)) == -8
    plan.destroy()
    p2.destroy()


@pytest.mark.slow
@pytest.mark.parametrize("name", ["j3d7pt_256x256x256_f64_T30", "j3d7pt_512x512x512_f64_T60",
                                  "j3d7pt_512x512x512_f32_T60"])
def test_3d_full_size_default_plan(name, capsys):
    """The benchmark's 3-D workloads in the plan it times (the default), whole grid, all steps, against the
    FP64 oracle (FP32: within its a priori bound, 2 (8T + 1) 2^-24 relative)."""
    w = inputs.workload(name)
    u0 = w.grid()
    npd = np.float64 if w.dtype == "f64" else np.float32
    with capsys.disabled():
        _say("3d full size", w.name)
        g = torch.from_numpy(u0.astype(npd)).to("cuda")
        plan = dtb.plan3d_for(g)
        desc = plan.describe()
        plan.run(g, w.coeffs, w.T)
        torch.cuda.synchronize()
        got = g.cpu().numpy()
        del g
        plan.destroy()
        ref = oracle_in_chunks(oracle.j3d7pt_f64, u0.astype(npd).astype(np.float64),
                               np.array(w.coeffs, dtype=npd).astype(np.float64), w.T, w.name, chunk=10)
    err = _err3(got, ref, w.cols)
    tol = TOL_F64 if w.dtype == "f64" else 2 * (8 * w.T + 1) * 2.0 ** -24
    record(workload=w.name, dtype=w.dtype, plan=desc, rel_max_err_vs_fp64_oracle=err, tolerance=tol)
    assert desc["path"] == dtb.PATH_STREAM3D and desc["stencil"] == 7
    assert err <= tol, err
