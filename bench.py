#!/usr/bin/env python3
"""Benchmark: j2d5pt under deep temporal blocking on one MI355X.

One "step" of this benchmark is one whole pass of the hot path over one
batch: dtb_run of the 16384 x 16384 FP64 grid for T = 2000 time steps (the
largest single-GPU FP64 configuration; the grid is larger than the chip, so the
tile-serial sweep runs it).  Throughput is counted in interior cell-updates:
rows * cols * T per step, divided by wall time.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu] [--no-extras]

Prints ONE JSON line.  Besides the headline value it carries:
  roofline        the DTB kernel's achieved FP64 arithmetic rate (9 flops per
                  cell-update: one multiply and four fused multiply-adds) against
                  the chip's FP64 vector peak; kernel duration from HIP events on
                  the launch stream; HBM traffic per launch from rocprofv3
                  counters while the kernel sources match the recorded hash;
  denominators    measured on the running part: LDS read/write bandwidth, copy
                  bandwidth from the Infinity Cache and from HBM, device-barrier
                  and neighbour-flag latency;
  baseline_1step  the untiled one-launch-per-time-step kernel on the same grid;
  cpu_baseline    the CPU oracle on a bounded sample of the same workload;
  other_configs   every other configuration at its full step count: median,
                  min and max of >= 5 runs, the one-step kernel beside it, the
                  error against the FP64 oracle recorded by the full-size parity
                  tests on the same kernel sources, and the roofline fractions;
                  and the 2048^2 and 8192^2 FP64 workloads under the three
                  synchronisation designs (neighbour flags, a device-wide
                  barrier per exchange, overlapped per-workgroup blocking).
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
PEAK_FP32_VECTOR_TFLOPS = 157.3  # with packed FP32; the kernels are built without it (78.6 unpacked)
PEAK_HBM_GBS = 8000.0
PEAK_LDS_TBS = 256 * 2.4e9 * 128 / 1e12  # datasheet LDS rate, 128 B per clock per CU
FLOPS_PER_UPDATE = 9      # j2d5pt: five products, four additions
FLOPS_PER_UPDATE9 = 17    # the 3 x 3 box: nine products, eight additions
FLOPS_PER_UPDATE3D = 13   # j3d7pt: seven products, six additions
HEADLINE = "j2d5pt_16384x16384_f64_T2000"

# HBM traffic per launch of the headline kernel (rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE, each scaled by the same counter on a plain copy of known size)
# and the full-size accuracy records (pytest with DTB_ACCURACY_LOG); both are
# used only while the kernel sources hash to the value recorded with them.
PROFILES = os.path.join(ROOT, "profiles")
ACCURACY_FILE = os.path.join(PROFILES, "accuracy_fullsize.md")


def _source_hash() -> str:
    from paper_2306_03336_amd import build
    return build.kernel_source_hash()


def _traffic_file(kernel: str, workload: str) -> str:
    return os.path.join(PROFILES, f"{kernel}_{workload}_traffic.md")


def _recorded_traffic(kernel: str, workload: str):
    """Bytes per launch recorded for this kernel and workload, if the kernel sources still match."""
    try:
        text = open(_traffic_file(kernel, workload)).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("workload") != workload or vals.get("kernel_source_sha256") != _source_hash():
        return None
    try:
        return int(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _accuracy_records():
    """Full-size accuracy records (JSON objects, one per bullet line) that match the current sources."""
    try:
        text = open(ACCURACY_FILE).read()
    except OSError:
        return []
    h = _source_hash()
    out = []
    for line in text.splitlines():
        line = line.strip()
        if line.startswith("- `{") and line.endswith("}`"):
            try:
                rec = json.loads(line[3:-1])
            except ValueError:
                continue
            if rec.get("kernel_source_sha256") == h:
                out.append(rec)
    return out


def _error_for(records, workload, dtype):
    for r in records:
        if r.get("workload") == workload and r.get("dtype") == dtype:
            keep = {k: v for k, v in r.items() if k not in ("plan", "exact_mode_plan", "kernel_source_sha256")}
            keep["source"] = "tests/test_gpu_fullsize.py / tests/test_gpu_parity.py, profiles/accuracy_fullsize.md"
            return keep
    return None


def _stats(ms_list, updates):
    import numpy as np
    ms = sorted(ms_list)
    med = float(np.median(ms))
    return {"reps": len(ms), "median_ms": round(med, 4), "min_ms": round(ms[0], 4), "max_ms": round(ms[-1], 4),
            "GCells_per_s": round(updates / (med / 1e3) / 1e9, 2),
            "GCells_per_s_min_max": [round(updates / (ms[-1] / 1e3) / 1e9, 2), round(updates / (ms[0] / 1e3) / 1e9, 2)]}


def _time_runs(run, torch, stream, reps):
    """Durations (ms) of `reps` calls of run(), HIP events on the launch stream around each."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(stream)
        run()
        e1.record(stream)
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in ev]


def _step_baseline(dtb, torch, stream, g, u0, coeffs, T, reps, stencil=5):
    """The untiled kernel: T launches of the one-step kernel, timed as launches (once) and as a HIP graph of
    the T launches (reps replays); the faster is the baseline."""
    sp = dtb.plan_for(g, T, path=dtb.PATH_STEP, stencil=stencil)
    g.copy_(u0)
    sp.run(g, coeffs, min(T, 200))
    torch.cuda.synchronize()
    launches = _time_runs(lambda: sp.run(g, coeffs, T), torch, stream, 1)[0]
    graph_ms = None
    try:
        side = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                sp.run(g, coeffs, T, stream=side)
        graph.replay()
        torch.cuda.synchronize()
        graph_ms = _time_runs(graph.replay, torch, stream, reps)
        del graph
    except Exception as e:  # the launch-by-launch figure stands on its own
        print(f"[bench] step-kernel graph skipped: {type(e).__name__}: {e}", file=sys.stderr, flush=True)
    sp.destroy()
    return launches, graph_ms


def _lds_bytes_per_launch(desc, T, b):
    """LDS bytes a DTB launch moves, counted from the plan: every step each wave stores its top and bottom
    rows and loads its neighbours' (4 rows of ext_cols cells); every exchange moves the border strips
    (rim out, ring in) through the staging area, each cell written and read once (counted as 4 b per
    ring-or-rim cell, rim + ring <= 4 k (ext_rows + ext_cols))."""
    nwg, waves, ER, EC, k = desc["workgroups"], desc["waves"], desc["ext_rows"], desc["ext_cols"], desc["ghost_k"]
    tiles = max(1, desc["big_tiles"])
    per_step = nwg * waves * 4 * EC * b
    per_exchange = nwg * 4 * k * (ER + EC) * 4 * b
    # The sweep runs every big tile for all T steps (one after another), idle slots excluded only
    # approximately (every slot of the launch counted): an upper bound.
    return tiles * T * (per_step + per_exchange / max(k, 1))


def _denominators(dtb):
    """Measured: LDS bandwidth, copy bandwidth (MALL- and HBM-sized buffers), barrier and flag latency."""
    out = {}
    try:
        ms, byt = dtb.probe(dtb.PROBE_LDS_READ, iters=4096)
        out["lds_read_TBs"] = round(byt / (ms / 1e3) / 1e12, 2)
        ms, byt = dtb.probe(dtb.PROBE_LDS_WRITE, iters=4096)
        out["lds_write_TBs"] = round(byt / (ms / 1e3) / 1e12, 2)
        for label, size, iters in (("copy_64MiB", 64 << 20, 50), ("copy_4GiB", 4 << 30, 5)):
            ms, byt = dtb.probe(dtb.PROBE_COPY, size=size, iters=iters)
            out[label + "_GBs"] = round(byt / (ms / 1e3) / 1e9, 1)
        ms, n = dtb.probe(dtb.PROBE_BARRIER, iters=2000)
        out["grid_barrier_us"] = round(ms * 1e3 / n, 3)
        ms, n = dtb.probe(dtb.PROBE_FLAGS, iters=2000)
        out["neighbour_flags_us"] = round(ms * 1e3 / n, 3)
        out["note"] = ("LDS: 16 B per lane per access, conflict-free, 2 workgroups per CU; copy: 16 B per lane, "
                       "bytes read + written; barrier: two-level device barrier over one workgroup per CU; "
                       "flags: raise own flag, wait for 8 neighbours, one workgroup per CU")
    except Exception as e:
        out["error"] = f"{type(e).__name__}: {e}"
    return out


def _rooflines(gc, dtype, desc, T, updates, dtb_ms, den, flops=FLOPS_PER_UPDATE):
    b = 8 if dtype == "f64" else 4
    peak = PEAK_FP64_VECTOR_TFLOPS if dtype == "f64" else PEAK_FP32_VECTOR_TFLOPS
    tflops = flops * gc / 1e3
    r = {"valu_TFLOPs": round(tflops, 3), "valu_peak_TFLOPs": peak, "frac_of_valu_peak": round(tflops / peak, 4),
         "frac_of_untiled_hbm_roofline": round(gc / (PEAK_HBM_GBS / (2 * b)), 3)}
    if desc is not None and desc.get("path") in (2, 3):
        lds = _lds_bytes_per_launch(desc, T, b)
        rate = lds / (dtb_ms / 1e3) / 1e12
        r["lds_bytes_per_cell_update"] = round(lds / updates, 3)
        r["lds_TBs"] = round(rate, 3)
        meas = den.get("lds_read_TBs") and den.get("lds_write_TBs")
        if meas:
            r["frac_of_measured_lds_bandwidth"] = round(rate / ((den["lds_read_TBs"] + den["lds_write_TBs"]) / 2), 4)
        r["frac_of_datasheet_lds_bandwidth"] = round(rate / PEAK_LDS_TBS, 4)
    return r


def _same_size_copy_GBs(torch, stream, like, launches=20):
    """Copy rate of a plain elementwise copy of a buffer the size of `like`, one launch per copy, launches
    back to back (what a one-step kernel does each step: read the grid once, write it once): bytes read and
    written per launch over the median launch time."""
    src = torch.ones_like(like)
    dst = torch.empty_like(like)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    ms = _time_runs(lambda: torch.mul(src, 1.0, out=dst), torch, stream, launches)
    ms.sort()
    med = ms[len(ms) // 2]
    nbytes = 2 * like.numel() * like.element_size()
    del src, dst
    return round(nbytes / (med / 1e3) / 1e9, 1)


def _one_config(dtb, inputs, torch, np, stream, name, records, den, reps=5):
    w = inputs.workload(name)
    dt = torch.float64 if w.dtype == "f64" else torch.float32
    u0 = torch.from_numpy(w.grid()).to(device="cuda", dtype=dt)
    g = u0.clone()
    plan = dtb.plan_for(g, w.T, stencil=w.pts)
    plan.run(g, w.coeffs, w.T)       # warm-up
    plan.check()
    g.copy_(u0)
    ms = _time_runs(lambda: plan.run(g, w.coeffs, w.T), torch, stream, reps)
    plan.check()
    d = plan.describe()
    plan.destroy()
    launches, graph_ms = _step_baseline(dtb, torch, stream, g, u0, w.coeffs, w.T, reps, w.pts)
    same_copy = _same_size_copy_GBs(torch, stream, u0)
    del g, u0
    torch.cuda.empty_cache()
    updates = w.cell_updates
    st = _stats(ms, updates)
    b = 8 if w.dtype == "f64" else 4
    if graph_ms:
        base = _stats(graph_ms, updates)
        base["variant"] = "HIP graph of the T launches"
        if launches < base["median_ms"]:
            base = _stats([launches], updates)
            base["variant"] = "T stream launches"
    else:
        base = _stats([launches], updates)
        base["variant"] = "T stream launches"
    base["launches"] = w.T
    base["achieved_GBs_algorithmic"] = round(base["GCells_per_s"] * 2 * b, 1)
    copy_key = "copy_64MiB_GBs" if 2 * (w.rows + 2) * (w.cols + 2) * b <= 256 << 20 else "copy_4GiB_GBs"
    if den.get(copy_key):
        base["frac_of_measured_copy_bandwidth"] = round(base["achieved_GBs_algorithmic"] / den[copy_key], 3)
        base["copy_reference"] = copy_key
    base["same_size_copy_per_launch_GBs"] = same_copy
    base["frac_of_same_size_copy"] = round(base["achieved_GBs_algorithmic"] / same_copy, 3)
    return {"workload": name, "dtype": w.dtype, "T": w.T, "cell_updates": updates, "plan": d, "dtb": st,
            "step_kernel": base, "dtb_speedup": round(base["median_ms"] / st["median_ms"], 3),
            "roofline": _rooflines(st["GCells_per_s"], w.dtype, d, w.T, updates, st["median_ms"], den,
                                   FLOPS_PER_UPDATE9 if w.pts == 9 else FLOPS_PER_UPDATE),
            "error_vs_oracle": _error_for(records, name, w.dtype)}


def _batched(dtb, inputs, torch, np, stream, records, reps=5):
    probs = inputs.batched_set(5)
    grids = []
    for p in probs:
        dt = torch.float64 if p.dtype == "f64" else torch.float32
        grids.append((torch.from_numpy(p.grid()).to(device="cuda", dtype=dt), p.coeffs, p.T))
    updates = sum(p.cell_updates for p in probs)
    dtb.run_batched(grids)          # plans, allocates, builds the graph
    dtb.batch_check()
    ms = _time_runs(lambda: dtb.run_batched(grids), torch, stream, reps)   # graph replays
    dtb.batch_check()
    # The same grids one at a time through dtb_run (cached plans, built in a first pass).
    for g, c, T in grids:
        dtb.run(g, c, 1)
    torch.cuda.synchronize()

    def one_at_a_time():
        for g, c, T in grids:
            dtb.run(g, c, T)
    ms1 = _time_runs(one_at_a_time, torch, stream, reps)
    st, st1 = _stats(ms, updates), _stats(ms1, updates)
    return {"workload": "j2d5pt_batch64_seed5", "grids": len(probs), "cell_updates": updates, "dtb_batched": st,
            "one_at_a_time": st1, "batched_speedup": round(st1["median_ms"] / st["median_ms"], 3),
            "error_vs_oracle": _error_for(records, "j2d5pt_batch64_seed5", "f64+f32")}


def _designs(dtb, inputs, torch, np, stream, name, reps=5):
    """The same workload under the synchronisation designs the paper weighs: neighbour epoch flags (the
    default), a device-wide barrier at every exchange (Section 3.2 as printed; resident grids only), and
    overlapped per-workgroup blocking with no synchronisation between workgroups (Section 2)."""
    w = inputs.workload(name)
    dt = torch.float64 if w.dtype == "f64" else torch.float32
    u0 = torch.from_numpy(w.grid()).to(device="cuda", dtype=dt)
    g = u0.clone()
    out = {"workload": name}
    variants = [("neighbour_flags", {}), ("grid_barrier", dict(path=dtb.PATH_RESIDENT, sync=dtb.SYNC_GRID_BARRIER)),
                ("overlapped", dict(path=dtb.PATH_OVERLAPPED))]
    for label, opts in variants:
        try:
            plan = dtb.plan_for(g, w.T, **opts)
        except dtb.DtbError as e:
            if label == "grid_barrier":
                # A grid larger than the chip is swept: big tiles already meet at a device-wide barrier;
                # an exchange barrier inside a big tile is offered for resident grids only.
                out[label] = {"not_applicable": "grid larger than the chip (tile-serial sweep)", "status": str(e)}
            else:
                out[label] = {"error": str(e)}
            continue
        g.copy_(u0)
        plan.run(g, w.coeffs, w.T)
        plan.check()
        ms = _time_runs(lambda: plan.run(g, w.coeffs, w.T), torch, stream, reps)
        plan.check()
        out[label] = {"plan": plan.describe(), **_stats(ms, w.cell_updates)}
        plan.destroy()
    base = out.get("neighbour_flags", {}).get("median_ms")
    for label, _ in variants[1:]:
        if base and "median_ms" in out.get(label, {}):
            out[label]["time_vs_neighbour_flags"] = round(out[label]["median_ms"] / base, 3)
    del g, u0
    torch.cuda.empty_cache()
    return out


def _one_config3(dtb, inputs, torch, np, stream, name, records, den, reps=5):
    """A j3d7pt workload: the default streaming plan against the fastest one-step-per-launch form (the
    one-step kernel as T launches or one HIP graph of them, and the streaming kernel with K = 1), all timed
    with HIP events on the launch stream."""
    w = inputs.workload(name)
    dt = torch.float64 if w.dtype == "f64" else torch.float32
    u0 = torch.from_numpy(w.grid()).to(device="cuda", dtype=dt)
    g = u0.clone()
    plan = dtb.plan3d_for(g)
    plan.run(g, w.coeffs, w.T)
    torch.cuda.synchronize()
    g.copy_(u0)
    ms = _time_runs(lambda: plan.run(g, w.coeffs, w.T), torch, stream, reps)
    d = plan.describe()
    plan.destroy()
    sp = dtb.plan3d_for(g, path=dtb.PATH_STEP)
    sp.run(g, w.coeffs, w.T)
    torch.cuda.synchronize()
    launches = _time_runs(lambda: sp.run(g, w.coeffs, w.T), torch, stream, 3)
    graph_ms = None
    try:
        side = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                sp.run(g, w.coeffs, w.T, stream=side)
        graph.replay()
        torch.cuda.synchronize()
        graph_ms = _time_runs(graph.replay, torch, stream, 3)
        del graph
    except Exception as e:
        print(f"[bench] 3-D step-kernel graph skipped: {type(e).__name__}: {e}", file=sys.stderr, flush=True)
    sp.destroy()
    # The streaming kernel advancing one step per launch (1-deep rings, T launches): also HBM to HBM every
    # step, and the faster one-step form in FP64.
    k1 = dtb.plan3d_for(g, ghost_k=1)
    k1.run(g, w.coeffs, w.T)
    torch.cuda.synchronize()
    k1_ms = _time_runs(lambda: k1.run(g, w.coeffs, w.T), torch, stream, 3)
    k1.destroy()
    del g, u0
    torch.cuda.empty_cache()
    updates = w.cell_updates
    b = 8 if w.dtype == "f64" else 4
    st = _stats(ms, updates)
    base = _stats(launches, updates)
    base["variant"] = "one-step kernel, T stream launches"
    if graph_ms and float(np.median(graph_ms)) < base["median_ms"]:
        base = _stats(graph_ms, updates)
        base["variant"] = "one-step kernel, HIP graph of the T launches"
    if float(np.median(k1_ms)) < base["median_ms"]:
        base = _stats(k1_ms, updates)
        base["variant"] = "streaming kernel with K = 1, T launches"
    base["launches"] = w.T
    base["achieved_GBs_algorithmic"] = round(base["GCells_per_s"] * 2 * b, 1)
    if den.get("copy_4GiB_GBs"):
        base["frac_of_measured_copy_bandwidth"] = round(base["achieved_GBs_algorithmic"] / den["copy_4GiB_GBs"], 3)
        base["copy_reference"] = "copy_4GiB_GBs"
    peak = PEAK_FP64_VECTOR_TFLOPS if w.dtype == "f64" else PEAK_FP32_VECTOR_TFLOPS
    tflops = FLOPS_PER_UPDATE3D * st["GCells_per_s"] / 1e3
    return {"workload": name, "dtype": w.dtype, "T": w.T, "cell_updates": updates, "plan": d, "dtb": st,
            "step_kernel": base, "dtb_speedup": round(base["median_ms"] / st["median_ms"], 3),
            "roofline": {"valu_TFLOPs": round(tflops, 3), "valu_peak_TFLOPs": peak,
                         "frac_of_valu_peak": round(tflops / peak, 4),
                         "frac_of_untiled_hbm_roofline": round(st["GCells_per_s"] / (PEAK_HBM_GBS / (2 * b)), 3)},
            "error_vs_oracle": _error_for(records, name, w.dtype)}


SECONDARY = [("cfg1_256_f64", "j2d5pt_256x256_f64_T16", 100),
             ("cfg2_2048_f64_resident", "j2d5pt_2048x2048_f64_T10000", 5),
             ("cfg3_8192_f64_sweep", "j2d5pt_8192x8192_f64_T1000", 5),
             ("cfg4a_3072_f32_resident", "j2d5pt_3072x3072_f32_T2000", 5),
             ("cfg4a_3072_f64_sweep", "j2d5pt_3072x3072_f64_T2000", 5),
             ("cfg4b_16384_f32_sweep", "j2d5pt_16384x16384_f32_T2000", 5),
             ("cfg6_box_2048_f64_sweep", "j2d9pt_2048x2048_f64_T10000", 5),
             ("cfg7_box_8192_f64_sweep", "j2d9pt_8192x8192_f64_T1000", 5),
             ("cfg7_box_8192_f32_sweep", "j2d9pt_8192x8192_f32_T1000", 5),
             ("cfg8_3d_512_f64_stream", "j3d7pt_512x512x512_f64_T60", 5),
             ("cfg8_3d_512_f32_stream", "j3d7pt_512x512x512_f32_T60", 5)]


def _extras(dtb, inputs, torch, np, stream, records, den, skip):
    out = {}
    jobs = [(key, (lambda n=name, r=reps: (_one_config3 if n.startswith("j3d7pt") else _one_config)(
                dtb, inputs, torch, np, stream, n, records, den, r)))
            for key, name, reps in SECONDARY if name != skip]
    jobs.append(("cfg5_batch64", lambda: _batched(dtb, inputs, torch, np, stream, records)))
    jobs.append(("designs_2048_f64", lambda: _designs(dtb, inputs, torch, np, stream, "j2d5pt_2048x2048_f64_T10000")))
    jobs.append(("designs_8192_f64", lambda: _designs(dtb, inputs, torch, np, stream, "j2d5pt_8192x8192_f64_T1000")))
    jobs.append(("designs_16384_f64",
                 lambda: _designs(dtb, inputs, torch, np, stream, "j2d5pt_16384x16384_f64_T2000", reps=3)))
    for key, fn in jobs:
        print(f"[bench] {key}", file=sys.stderr, flush=True)
        try:
            out[key] = fn()
        except Exception as e:  # a secondary configuration must not hide the headline line
            out[key] = {"error": f"{type(e).__name__}: {e}"}
    return out


def _cpu_baseline(w, budget_s: float):
    """Time the CPU oracle on a bounded number of steps of the same grid."""
    import oracle  # test infrastructure, used only for this leg
    u = w.grid()
    nt = oracle.default_threads()
    fn = oracle.j2d9pt_f64 if w.pts == 9 else oracle.j2d5pt_f64
    steps, t0 = 0, time.perf_counter()
    chunk = max(1, min(50, int(2e9 // (w.rows * w.cols))))
    while time.perf_counter() - t0 < budget_s and steps < w.T:
        u = fn(u, w.coeffs, chunk, nthreads=nt)
        steps += chunk
    dt = time.perf_counter() - t0
    u1 = w.grid()
    s1, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < budget_s / 4 and s1 < w.T:
        u1 = fn(u1, w.coeffs, 1, nthreads=1)
        s1 += 1
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(w.rows * w.cols * steps / dt / 1e9, 4), "unit": "GCells/s", "cores": nt,
            "kind": "oracle",
            "sample": f"{w.rows}x{w.cols} FP64, {steps} of the {w.T} time steps ({dt:.1f} s, {nt} threads)",
            "one_thread_value": round(w.rows * w.cols * s1 / dt1 / 1e9, 4),
            "one_thread_sample": f"{s1} steps ({dt1:.1f} s)", "host_cpu": model, "host_cpus": os.cpu_count()}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-step-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary configurations")
    ap.add_argument("--no-probes", action="store_true", help="skip the micro-benchmarks of the denominators")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed region, copy a buffer of this many MiB three times with an "
                         "elementwise kernel (a plain copy of known size, to scale hardware byte counters)")
    ap.add_argument("--source-hash", action="store_true", help="print the kernel source hash and exit")
    ap.add_argument("--phase-clocks", action="store_true",
                    help="after the timed region, run the workload once more with per-workgroup phase clocks "
                         "and report the time per step spent in steps and in each exchange phase")
    args = ap.parse_args()
    if args.source_hash:
        print(_source_hash())
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(a multi-GPU layout is not implemented)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2306_03336_amd import dtb, inputs

    w = inputs.workload(args.workload)
    if w.pts == 7:
        # A j3d7pt workload on its own (for profiling): its default streaming plan, the same record as in
        # other_configs, printed as one JSON line; optionally the copy probe that scales the byte counters.
        stream = torch.cuda.current_stream()
        r = _one_config3(dtb, inputs, torch, np, stream, w.name, _accuracy_records(), {}, max(1, args.steps))
        if args.copy_probe_mb > 0:
            n = args.copy_probe_mb * (1 << 20) // 8
            a = torch.ones(n, dtype=torch.float64, device="cuda")
            bb = torch.empty_like(a)
            for _ in range(3):
                torch.mul(a, 1.0, out=bb)
            torch.cuda.synchronize()
        print(json.dumps({"metric": "GCells/s j3d7pt, 2.5D streaming vs 1-step kernel on 1 MI355X",
                          "value": r["dtb"]["GCells_per_s"], "unit": "GCells/s", "n_gpus": 1,
                          "steps": max(1, args.steps), "higher_is_better": True, "dtype": w.dtype,
                          "data": "synthetic", "config": {"workload": w.name, "depth": w.depth, "rows": w.rows,
                                                          "cols": w.cols, "T": w.T}, "detail": r}))
        return 0
    dt = torch.float64 if w.dtype == "f64" else torch.float32
    u0 = torch.from_numpy(w.grid()).to(device="cuda", dtype=dt)
    g = u0.clone()
    stream = torch.cuda.current_stream()
    plan = dtb.plan_for(g, w.T, stencil=w.pts)
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
    updates = w.cell_updates
    value = updates * args.steps / wall / 1e9
    print(f"[bench] timed {args.steps} runs: {value:.1f} GCells/s", file=sys.stderr, flush=True)

    base = None
    if not args.no_step_baseline:
        launches, graph_ms = _step_baseline(dtb, torch, stream, g, u0, w.coeffs, w.T, 3, w.pts)
        bms = min([launches] + (graph_ms or []))
        bval = updates / (bms / 1e3) / 1e9
        b = 8 if w.dtype == "f64" else 4
        base = {"value": round(bval, 3), "unit": "GCells/s", "ms_per_run": round(bms, 3),
                "ms_per_run_launches": round(launches, 3),
                "ms_per_run_graph": None if not graph_ms else [round(x, 3) for x in graph_ms],
                "launches": w.T, "dtb_speedup": round(value / bval, 3),
                "hbm_roofline_GCells": PEAK_HBM_GBS / (2 * b),
                "achieved_GBs_algorithmic": round(bval * 2 * b, 1)}
        same = _same_size_copy_GBs(torch, stream, u0)
        base["same_size_copy_per_launch_GBs"] = same
        base["frac_of_same_size_copy"] = round(base["achieved_GBs_algorithmic"] / same, 3)
        print(f"[bench] one-step kernel: {bval:.1f} GCells/s", file=sys.stderr, flush=True)

    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        bb = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=bb)  # an elementwise kernel: reads and writes the buffer once each
        torch.cuda.synchronize()
        print(f"[bench] copy probe: 3 copies of {args.copy_probe_mb} MiB", file=sys.stderr, flush=True)
        del a, bb

    den = {} if args.no_probes else _denominators(dtb)
    records = _accuracy_records()

    peak = PEAK_FP64_VECTOR_TFLOPS if w.dtype == "f64" else PEAK_FP32_VECTOR_TFLOPS
    flops = FLOPS_PER_UPDATE9 if w.pts == 9 else FLOPS_PER_UPDATE
    achieved = flops * updates / (avg_ms / 1e3) / 1e12
    kname = {2: "k_dtb", 3: "k_dtb_sweep"}.get(desc["path"], "k_step")
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": _recorded_traffic(kname, w.name),
            "kernel": kname, "avg_launch_ms": round(avg_ms, 4),
            "launch_ms_min_median_max": [round(min(kern_ms), 4), round(float(np.median(kern_ms)), 4),
                                         round(max(kern_ms), 4)],
            "algorithmic_flops_per_launch": flops * updates}
    context = _rooflines(value, w.dtype, desc, w.T, updates, avg_ms, den, flops)
    context["error_vs_oracle"] = _error_for(records, w.name, w.dtype)

    phases = None
    if args.phase_clocks:
        # Where a step's time goes, from per-workgroup phase clocks of the same plan shape.
        tp = dtb.plan_for(g, w.T, debug=dtb.DEBUG_TIMING, stencil=w.pts)
        g.copy_(u0)
        tp.run(g, w.coeffs, w.T)
        tp.check()
        clocks = tp.timing()
        tp.destroy()
        keys = ("steps", "stage_out", "publish", "wait", "stage_in", "ghost", "total")
        phases = {k: round(float(np.mean([c[k] for c in clocks])) / w.T, 4) for k in keys}
        phases["unit"] = "us per time step, mean over workgroups"
        phases["exchanges"] = int(max(c["exchanges"] for c in clocks))
    plan.destroy()
    del g, u0
    torch.cuda.empty_cache()

    extras = {}
    if not args.no_extras:
        extras = _extras(dtb, inputs, torch, np, stream, records, den, w.name)

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
        "denominators": den,
        "phase_clocks": phases,
        "baseline_1step": base,
        "cpu_baseline": cpu,
        "other_configs": extras,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    rc = main()
    if rc:
        sys.exit(rc)
