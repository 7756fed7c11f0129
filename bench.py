#!/usr/bin/env python3
"""Benchmark: j2d5pt under deep temporal blocking on one MI355X.

One "step" of this benchmark is one whole pass of the hot path over one
batch: dtb_run of the 2048 x 2048 FP64 grid for T = 10000 time steps (the
grid stays on chip for all of them).  Throughput is counted in interior
cell-updates: rows * cols * T per step, divided by wall time.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu] [--no-step-baseline]

Prints ONE JSON line.  Besides the headline value it carries:
  roofline      the DTB kernel's achieved FP64 arithmetic rate (9 flops per
                cell-update: one multiply and four fused multiply-adds)
                against the chip's FP64 vector peak; duration from HIP events
                on the launch stream;
  baseline_1step  the untiled one-launch-per-time-step kernel on the same
                grid (T launches, HBM/Infinity-Cache bound), and DTB's speedup;
  cpu_baseline  the CPU oracle on a bounded sample of the same workload;
  other_configs the FP32 precision pair (3072^2 resident, 16384^2 swept for
                400 of its 2000 steps), the 8192^2 FP64 tile-serial sweep, and
                the 64-grid batch in one graph-replayed launch against the
                same grids run one at a time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR_TFLOPS = 78.6   # MI355X FP64 vector (FMA counted as 2 flops)
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
FLOPS_PER_UPDATE = 9

# HBM traffic of k_dtb per launch, measured with rocprofv3 --pmc (FETCH_SIZE,
# WRITE_SIZE, scaled by the same counters on a plain copy of known size); the
# figure is reported only while the kernel sources hash to the value recorded
# beside it.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_dtb_j2d5pt_2048x2048_f64_T10000_traffic.md")


def _kernel_source_hash() -> str:
    import hashlib
    csrc = os.path.join(ROOT, "paper_2306_03336_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def _recorded_traffic(workload: str):
    """(bytes per launch, source hash) recorded for this workload, if the sources still match."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("workload") != workload or vals.get("kernel_source_sha256") != _kernel_source_hash():
        return None
    try:
        return int(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _cpu_baseline(w, budget_s: float):
    """Time the CPU oracle on a bounded number of steps of the same grid."""
    import oracle  # test infrastructure, used only for this leg
    u = w.grid()
    nt = oracle.default_threads()
    steps, t0 = 0, time.perf_counter()
    chunk = 50
    while time.perf_counter() - t0 < budget_s and steps < w.T:
        u = oracle.j2d5pt_f64(u, w.coeffs, chunk, nthreads=nt)
        steps += chunk
    dt = time.perf_counter() - t0
    # One thread, a shorter sample of the same grid.
    u1 = w.grid()
    s1, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < budget_s / 4 and s1 < w.T:
        u1 = oracle.j2d5pt_f64(u1, w.coeffs, 10, nthreads=1)
        s1 += 10
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(w.rows * w.cols * steps / dt / 1e9, 4), "unit": "GCells/s", "cores": nt,
            "kind": "oracle",
            "sample": f"{w.rows}x{w.cols} FP64, {steps} of the {w.T} time steps ({dt:.1f} s, FP64, {nt} threads)",
            "one_thread_value": round(w.rows * w.cols * s1 / dt1 / 1e9, 4),
            "one_thread_sample": f"{s1} steps ({dt1:.1f} s)", "host_cpu": model, "host_cpus": os.cpu_count()}


def _time_run(plan, g, coeffs, T, torch, stream, reps=1):
    """Best of `reps` runs of T steps, milliseconds (HIP events on the launch stream)."""
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.run(g, coeffs, T)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    plan.check()
    return best


def _one_config(dtb, inputs, torch, np, stream, name, T=None, warm=50):
    w = inputs.workload(name)
    dt = torch.float64 if w.dtype == "f64" else torch.float32
    g = torch.from_numpy(w.grid()).to(device="cuda", dtype=dt)
    T = w.T if T is None else T
    plan = dtb.plan_for(g, w.T)
    plan.run(g, w.coeffs, min(warm, T))
    torch.cuda.synchronize()
    ms = _time_run(plan, g, w.coeffs, T, torch, stream)
    d = plan.describe()
    plan.destroy()
    # The one-step-per-launch kernel on the same grid and step count.
    sp = dtb.plan_for(g, T, path=dtb.PATH_STEP)
    sp.run(g, w.coeffs, min(warm, T))
    torch.cuda.synchronize()
    sms = _time_run(sp, g, w.coeffs, T, torch, stream)
    sp.destroy()
    del g
    torch.cuda.empty_cache()
    gc = w.rows * w.cols * T / (ms / 1e3) / 1e9
    sgc = w.rows * w.cols * T / (sms / 1e3) / 1e9
    b = 8 if w.dtype == "f64" else 4
    return {"workload": name, "dtype": w.dtype, "T_timed": T, "ms": round(ms, 3), "GCells_per_s": round(gc, 2),
            "step_kernel_GCells_per_s": round(sgc, 2), "dtb_speedup": round(gc / sgc, 3),
            "frac_of_untiled_hbm_roofline": round(gc / (PEAK_HBM_GBS / (2 * b)), 3), "plan": d}


def _batched(dtb, inputs, torch, np, stream):
    probs = inputs.batched_set(5)
    grids = []
    for p in probs:
        dt = torch.float64 if p.dtype == "f64" else torch.float32
        grids.append((torch.from_numpy(p.grid()).to(device="cuda", dtype=dt), p.coeffs, p.T))
    updates = sum(p.cell_updates for p in probs)
    dtb.run_batched(grids)          # plans, allocates, builds the graph
    dtb.batch_check()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    dtb.run_batched(grids)          # graph replay
    e1.record(stream)
    torch.cuda.synchronize()
    dtb.batch_check()
    ms = e0.elapsed_time(e1)
    # The same grids one at a time through dtb_run (cached plans, built in a first pass).
    for g, c, T in grids:
        dtb.run(g, c, 1)
    torch.cuda.synchronize()
    e0.record(stream)
    for g, c, T in grids:
        dtb.run(g, c, T)
    e1.record(stream)
    torch.cuda.synchronize()
    ms1 = e0.elapsed_time(e1)
    return {"workload": "j2d5pt_batch64_seed5", "grids": len(probs), "cell_updates": updates,
            "ms": round(ms, 3), "GCells_per_s": round(updates / (ms / 1e3) / 1e9, 2),
            "one_at_a_time_ms": round(ms1, 3), "one_at_a_time_GCells_per_s": round(updates / (ms1 / 1e3) / 1e9, 2),
            "batched_speedup": round(ms1 / ms, 3)}


def _extras(dtb, inputs, torch, np, stream):
    out = {}
    jobs = [("fp32_resident_3072", lambda: _one_config(dtb, inputs, torch, np, stream, "j2d5pt_3072x3072_f32_T2000")),
            ("fp64_sweep_8192", lambda: _one_config(dtb, inputs, torch, np, stream, "j2d5pt_8192x8192_f64_T1000")),
            ("fp32_sweep_16384", lambda: _one_config(dtb, inputs, torch, np, stream, "j2d5pt_16384x16384_f32_T2000",
                                                     T=400)),
            ("batched_64", lambda: _batched(dtb, inputs, torch, np, stream))]
    for key, fn in jobs:
        print(f"[bench] {key}", file=sys.stderr, flush=True)
        try:
            out[key] = fn()
        except Exception as e:  # a secondary configuration must not hide the headline line
            out[key] = {"error": f"{type(e).__name__}: {e}"}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="j2d5pt_2048x2048_f64_T10000")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-step-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary configurations")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed region, copy a buffer of this many MiB three times with an "
                         "elementwise kernel (a plain copy of known size, to scale hardware byte counters)")
    ap.add_argument("--source-hash", action="store_true", help="print the kernel source hash and exit")
    ap.add_argument("--phase-clocks", action="store_true",
                    help="after the timed region, run the workload once more with per-workgroup phase clocks "
                         "and report the time per step spent in steps and in each exchange phase")
    args = ap.parse_args()
    if args.source_hash:
        print(_kernel_source_hash())
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(a multi-GPU layout is not implemented)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2306_03336_amd import dtb, inputs

    w = inputs.workload(args.workload)
    dt = torch.float64 if w.dtype == "f64" else torch.float32
    u0 = torch.from_numpy(w.grid()).to(device="cuda", dtype=dt)
    g = u0.clone()
    stream = torch.cuda.current_stream()
    plan = dtb.plan_for(g, w.T)
    desc = plan.describe()
    print(f"[bench] {w.name} plan {desc}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        g.copy_(u0)
        plan.run(g, w.coeffs, w.T)
    plan.check()
    torch.cuda.synchronize()

    # Timed region: K whole runs, each advancing the grid another T steps.
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[2 * i].record(stream)
        plan.run(g, w.coeffs, w.T)
        ev[2 * i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.check()
    kern_ms = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(args.steps)]
    avg_ms = float(np.mean(kern_ms))
    ms_per_step = wall * 1e3 / args.steps
    updates = w.rows * w.cols * w.T
    value = updates * args.steps / wall / 1e9

    # The untiled baseline on the same grid: T launches of the one-step kernel.
    base = None
    if not args.no_step_baseline:
        sp = dtb.plan_for(g, w.T, path=dtb.PATH_STEP)
        g.copy_(u0)
        sp.run(g, w.coeffs, 200)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sp.run(g, w.coeffs, w.T)
        e1.record(stream)
        torch.cuda.synchronize()
        bms_launch = e0.elapsed_time(e1)
        # The same T launches captured once in a HIP graph and replayed (no
        # per-launch host overhead); the faster of the two is the baseline.
        bms_graph = None
        try:
            side = torch.cuda.Stream()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.stream(side):
                with torch.cuda.graph(graph, stream=side):
                    sp.run(g, w.coeffs, w.T, stream=side)
            graph.replay()
            torch.cuda.synchronize()
            e0.record(stream)
            graph.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            bms_graph = e0.elapsed_time(e1)
            del graph
        except Exception as e:  # the launch-by-launch figure stands on its own
            print(f"[bench] step-kernel graph skipped: {type(e).__name__}: {e}", file=sys.stderr, flush=True)
        bms = min(bms_launch, bms_graph) if bms_graph is not None else bms_launch
        bval = updates / (bms / 1e3) / 1e9
        bytes_per_update = 2 * (8 if w.dtype == "f64" else 4)
        base = {"value": round(bval, 3), "unit": "GCells/s", "ms_per_run": round(bms, 3),
                "ms_per_run_launches": round(bms_launch, 3),
                "ms_per_run_graph": None if bms_graph is None else round(bms_graph, 3),
                "launches": w.T, "dtb_speedup": round(value / bval, 3),
                "hbm_roofline_GCells": PEAK_HBM_GBS / bytes_per_update,
                "achieved_GBs_algorithmic": round(bval * bytes_per_update, 1)}
        sp.destroy()

    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)  # an elementwise kernel: reads and writes the buffer once each
        torch.cuda.synchronize()
        print(f"[bench] copy probe: 3 copies of {args.copy_probe_mb} MiB", file=sys.stderr, flush=True)
        del a, b

    b = 8 if w.dtype == "f64" else 4
    # Context figures: the untiled kernel's HBM roofline (one read and one write
    # per cell-step) and the LDS roofline at one LDS read and write per
    # cell-step (128 B per clock per CU); the DTB kernel keeps its tile in
    # registers and is bound by neither.
    hbm_roof = PEAK_HBM_GBS / (2 * b)
    lds_roof = 256 * 2.4e9 * 128 / (2 * b) / 1e9
    context = {"untiled_hbm_roofline_GCells": hbm_roof, "frac_of_untiled_hbm_roofline": round(value / hbm_roof, 3),
               "lds_roofline_GCells": round(lds_roof, 1), "frac_of_lds_roofline": round(value / lds_roof, 3)}

    peak = PEAK_FP64_VECTOR_TFLOPS if w.dtype == "f64" else PEAK_FP32_VECTOR_TFLOPS
    achieved = FLOPS_PER_UPDATE * updates / (avg_ms / 1e3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": _recorded_traffic(w.name),
            "kernel": "k_dtb", "avg_launch_ms": round(avg_ms, 4),
            "launch_ms_min_median_max": [round(min(kern_ms), 4), round(float(np.median(kern_ms)), 4),
                                         round(max(kern_ms), 4)]}

    phases = None
    if args.phase_clocks:
        # Where a step's time goes, from per-workgroup phase clocks of the same plan shape.
        tp = dtb.plan_for(g, w.T, debug=dtb.DEBUG_TIMING)
        g.copy_(u0)
        tp.run(g, w.coeffs, w.T)
        tp.check()
        clocks = tp.timing()
        tp.destroy()
        keys = ("steps", "stage_out", "publish", "wait", "stage_in", "ghost", "total")
        phases = {k: round(float(np.mean([c[k] for c in clocks])) / w.T, 4) for k in keys}
        phases["unit"] = "us per time step, mean over workgroups"
        phases["exchanges"] = int(max(c["exchanges"] for c in clocks))

    extras = {}
    if not args.no_extras:
        extras = _extras(dtb, inputs, torch, np, stream)

    cpu = None if args.no_cpu else _cpu_baseline(w, args.cpu_budget)

    out = {
        "metric": "GCells/s j2d5pt, DTB vs 1-step kernel on 1 MI355X, FP64 (<=1e-13) and FP32",
        "value": round(value, 3),
        "unit": "GCells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "rows": w.rows, "cols": w.cols, "T": w.T, "halo": w.halo,
                   "weights": w.weights, "seed": w.seed, "plan": desc},
        "roofline": roof,
        "context": context,
        "phase_clocks": phases,
        "baseline_1step": base,
        "cpu_baseline": cpu,
        "other_configs": extras,
    }
    print(json.dumps(out))
    plan.destroy()
    return 0


if __name__ == "__main__":
    rc = main()
    if rc:
        sys.exit(rc)
