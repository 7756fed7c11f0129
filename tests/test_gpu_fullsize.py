"""Full-size parity: the benchmark's configurations, in the launch configuration the benchmark times,
against the CPU oracle over the whole grid and every time step.

* FP64 (default fused chain) within 1e-13 relative max-norm of the FP64 oracle.
* FP32 (default fused chain) against the FP64 oracle run on the FP64 inputs (the end-to-end error
  of the precision path: input, coefficient and arithmetic rounding), inside an a priori bound;
  and the same plan in exact mode bit for bit against the FP32 oracle.
* The 64-grid batch after a graph replay, every grid.

Each result is printed as a ``[result]`` line and, when the environment variable
``DTB_ACCURACY_LOG`` names a file, appended to it as one JSON object per line (with the hash of the
kernel sources it was measured on).
"""
import numpy as np
import pytest

import oracle
from paper_2306_03336_amd import dtb, inputs
from record import oracle_in_chunks, record as _record, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

TOL_F64 = 1e-13
U_F32 = 2.0 ** -24


def f32_bound(T):
    """A priori relative max-norm bound of the FP32 path against the FP64 oracle for non-negative
    weights summing to 1 (each step is a convex combination, so errors do not grow): at most five
    roundings per cell per step, one rounding of each input cell and of each weight (the latter
    acting once per step), doubled for safety: 2 (6T + 1) u."""
    return 2 * (6 * T + 1) * U_F32


def f32_abs_bound(T, ref_max):
    """The same bound in absolute form, with gradual underflow: a rounding in the subnormal range errs
    by at most half the subnormal spacing, 2^-150, in absolute terms (not relative), and convex steps
    do not amplify it; at most six such roundings per cell per step, doubled.  It is what applies when
    the exact result falls below FP32's normal range (strongly asymmetric weights wash the field out
    through a zero halo), where the relative max-norm of any FP32 result is 1."""
    return f32_bound(T) * ref_max + 2 * 6 * T * 2.0 ** -150


def _say(*a):
    say("[case]", *a)


def _gpu_run(u, coeffs, T, dtype, **opts):
    """Plan for u's shape (default options unless given), run T steps, return (result, plan description)."""
    g = torch.from_numpy(np.ascontiguousarray(u.astype(dtype))).to("cuda")
    plan = dtb.plan_for(g, T, **opts)
    plan.run(g, coeffs, T)
    plan.check()
    desc = plan.describe()
    plan.destroy()
    out = g.cpu().numpy()
    del g
    torch.cuda.empty_cache()
    return out, desc


def _same_plan_exact(desc):
    """Options that rebuild a plan's tiling in exact mode."""
    o = dict(path=desc["path"], rows_per_lane=desc["rows_per_lane"], ghost_k=desc["ghost_k"], exact=True)
    if desc["path"] == dtb.PATH_SWEEP:
        o["depth_D"] = desc["depth_D"]
    else:
        o["waves"] = desc["waves"]
    return o


def _check_precision_pair(name64, name):
    """FP64 and FP32 runs of one configuration (the same input) against one FP64 oracle run on the FP64
    inputs."""
    w = inputs.workload(name)
    assert inputs.workload(name64).seed == w.seed and inputs.workload(name64).coeffs == w.coeffs
    u0 = w.grid()
    assert np.array_equal(inputs.workload(name64).grid()[:8], u0[:8])
    _say("oracle f64", name)
    ref = oracle_in_chunks(oracle.j2d5pt_f64, u0, w.coeffs, w.T, name64)
    # FP64, default plan.
    _say("gpu f64", name)
    got, desc = _gpu_run(u0, w.coeffs, w.T, np.float64)
    err = oracle.rel_max_err(got, ref)
    _record(workload=name64, dtype="f64", plan=desc, rel_max_err_vs_fp64_oracle=err, tolerance=TOL_F64)
    assert err <= TOL_F64, (name, err)
    assert np.array_equal(got[0], u0[0]) and np.array_equal(got[:, 0], u0[:, 0])
    del got
    # FP32, default plan: the end-to-end error against the FP64 oracle on the FP64 inputs.
    _say("gpu f32", name)
    got32, desc32 = _gpu_run(u0, w.coeffs, w.T, np.float32)
    err32 = oracle.rel_max_err(got32, ref)
    del ref
    bound = f32_bound(w.T)
    # FP32 exact mode with the same tiling, bit for bit against the FP32 oracle.
    u32 = u0.astype(np.float32)
    del u0
    _say("oracle f32", name)
    ref32 = oracle_in_chunks(oracle.j2d5pt_f32, u32, w.coeffs, w.T, name)
    err_arith = oracle.rel_max_err(got32, ref32)
    del got32
    _say("gpu f32 exact", name, _same_plan_exact(desc32))
    ex32, dex = _gpu_run(u32, w.coeffs, w.T, np.float32, **_same_plan_exact(desc32))
    bitwise = bool(np.array_equal(ex32, ref32))
    _record(workload=name, dtype="f32", plan=desc32, rel_max_err_vs_fp64_oracle=err32, a_priori_bound=bound,
            rel_max_err_vs_fp32_oracle=err_arith, exact_mode_plan=dex, exact_mode_bitwise_vs_fp32_oracle=bitwise)
    for key in ("path", "rows_per_lane", "cols_per_lane", "ghost_k", "depth_D", "workgroups", "big_tiles"):
        assert dex[key] == desc32[key], (key, dex, desc32)
    assert bitwise, name
    assert 1e-9 < err32 <= bound, (name, err32, bound)


def test_precision_pair_3072_T2000(capsys):
    """3072^2, T = 2000, weights 0.2, halo 0: FP64 (does not fit on chip: swept) and FP32 (resident)."""
    with capsys.disabled():  # progress lines reach the terminal while the oracle runs
        _check_precision_pair("j2d5pt_3072x3072_f64_T2000", "j2d5pt_3072x3072_f32_T2000")


@pytest.mark.timeout(900)
def test_precision_pair_16384_T2000(capsys):
    """16384^2, T = 2000, weights 0.2, halo 0: FP64 and FP32, both swept, over all 2000 steps."""
    with capsys.disabled():
        _check_precision_pair("j2d5pt_16384x16384_f64_T2000", "j2d5pt_16384x16384_f32_T2000")


@pytest.mark.timeout(600)
def test_batch64_after_graph_replay(capsys):
    """The 64-grid batch (sides 128..3072, T 100..2000, FP64 and FP32 alternating): the first call plans and
    captures, the second replays the graph on freshly reset grids; every grid against the oracle."""
    with capsys.disabled():
        _batch64()


def _batch64():
    probs = inputs.batched_set(5)
    grids = []
    for p in probs:
        dt = torch.float64 if p.dtype == "f64" else torch.float32
        grids.append((torch.from_numpy(p.grid()).to(device="cuda", dtype=dt), p.coeffs, p.T))
    init = [g.clone() for g, _, _ in grids]
    _say("batch64 first call")
    dtb.run_batched(grids)
    dtb.batch_check()
    for (g, _, _), g0 in zip(grids, init):
        g.copy_(g0)
    _say("batch64 graph replay")
    dtb.run_batched(grids)
    dtb.batch_check()
    worst = {"f64": 0.0, "f32": 0.0}
    underflowed = []
    tiny = float(np.finfo(np.float32).tiny)
    for p, (g, coeffs, T) in zip(probs, grids):
        u = p.grid()
        got = g.cpu().numpy()
        if p.dtype == "f64":
            ref = oracle.j2d5pt_f64(u, coeffs, T)
            err = oracle.rel_max_err(got, ref)
            assert err <= TOL_F64, (p.index, p.side, p.T, p.dtype, err)
        else:
            # FP32 grid: the FP64 oracle on the same float-rounded input and coefficients.
            ref = oracle.j2d5pt_f64(u.astype(np.float32).astype(np.float64),
                                    np.array(coeffs, dtype=np.float32).astype(np.float64), T)
            err = oracle.rel_max_err(got, ref)
            ref_max = float(np.max(np.abs(ref[1:-1, 1:-1])))
            abs_err = float(np.max(np.abs(got[1:-1, 1:-1].astype(np.float64) - ref[1:-1, 1:-1])))
            assert abs_err <= f32_abs_bound(T, ref_max), (p.index, p.side, p.T, abs_err, ref_max)
            if ref_max < tiny:
                underflowed.append((p.index, p.side, p.T, ref_max))
                say(f"[result] batch grid {p.index}: exact result below FP32's normal range "
                    f"(max {ref_max:.3e}); FP32 max |u| {float(np.max(np.abs(got))):.3e}")
                continue
            assert err <= f32_bound(T), (p.index, p.side, p.T, p.dtype, err)
        say(f"[result] batch grid {p.index}: {p.side}^2 {p.dtype} T={T} rel max err {err:.3e}")
        worst[p.dtype] = max(worst[p.dtype], err)
    _record(workload="j2d5pt_batch64_seed5", dtype="f64+f32", grids=len(probs),
            worst_rel_max_err_f64=worst["f64"], worst_rel_max_err_f32=worst["f32"],
            f32_reference="FP64 oracle on the float-rounded inputs and coefficients",
            f32_grids_below_normal_range=len(underflowed))
