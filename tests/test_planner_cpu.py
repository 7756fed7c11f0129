"""The resident-path tile planner, run on the host without a GPU (dtb_test_layout).

Checks, for many shapes: owned regions tile the interior exactly; each tile's
k-deep fresh ring lies inside its register tile; register tiles stay inside
the storage; neighbour lists are exactly the tiles within k (and symmetric);
XCD grouping keeps most exchanges inside one XCD.
"""
import itertools

import numpy as np
import pytest

from paper_2306_03336_amd import dtb

SHAPES = [(1, 1), (1, 200), (200, 1), (127, 131), (256, 256), (300, 129), (129, 257), (1000, 777),
          (2048, 2048), (3072, 3072)]
INSTANCES = [(8, 2, 8), (16, 2, 8), (24, 2, 8), (16, 4, 8), (24, 4, 8)]  # rows/lane, cols/lane, waves


def _check_layout(rows, cols, R, C, waves, k, lay):
    ER, EC = waves * R, 64 * C
    owner = np.full((rows + 2, cols + 2), -1, dtype=np.int64)
    for a, d in enumerate(lay):
        assert 1 <= d["own_r0"] < d["own_r1"] <= rows + 1 and 1 <= d["own_c0"] < d["own_c1"] <= cols + 1
        blk = owner[d["own_r0"]:d["own_r1"], d["own_c0"]:d["own_c1"]]
        assert np.all(blk == -1), "owned regions overlap"
        blk[...] = a
        # fresh ring inside the register tile
        f_r0, f_r1 = max(d["own_r0"] - k, 1), min(d["own_r1"] + k, rows + 1)
        f_c0, f_c1 = max(d["own_c0"] - k, 1), min(d["own_c1"] + k, cols + 1)
        assert d["ext_r0"] <= f_r0 and f_r1 <= d["ext_r0"] + ER
        assert d["ext_c0"] <= f_c0 and f_c1 <= d["ext_c0"] + EC
        assert d["ext_r0"] >= 1 and d["ext_c0"] >= 1
        if not d["narrow_rows"]:
            assert d["ext_r0"] + ER - 1 <= rows
        if not d["narrow_cols"]:
            assert d["ext_c0"] + EC - 1 <= cols
        assert d["narrow_rows"] == (rows < ER) and d["narrow_cols"] == (cols < EC)
    assert np.all(owner[1:rows + 1, 1:cols + 1] >= 0), "interior not covered"
    for a, d in enumerate(lay):
        f = owner[max(d["own_r0"] - k, 1):min(d["own_r1"] + k, rows + 1),
                  max(d["own_c0"] - k, 1):min(d["own_c1"] + k, cols + 1)]
        want = sorted(set(np.unique(f).tolist()) - {a})
        assert sorted(d["nb"]) == want
    for a, d in enumerate(lay):
        for b in d["nb"]:
            assert a in lay[b]["nb"]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("inst", INSTANCES, ids=lambda i: f"R{i[0]}C{i[1]}")
@pytest.mark.parametrize("k", [1, 2, 5, 8, 16])
def test_layout_properties(shape, inst, k):
    rows, cols = shape
    R, C, waves = inst
    lay = dtb.test_layout(rows, cols, R, C, waves, k, 8, max_wg=8192)
    if lay is None:
        # only impossible when the ghost ring does not fit the register tile
        assert 2 * k >= min(waves * R, 64 * C) and (rows > waves * R or cols > 64 * C)
        return
    _check_layout(rows, cols, R, C, waves, k, lay)


def test_config_2048_fits_one_wave_of_workgroups():
    lay = dtb.test_layout(2048, 2048, 24, 2, 8, 8)
    assert lay is not None and len(lay) <= 256


def test_xcd_grouping_keeps_exchanges_local():
    lay = dtb.test_layout(2048, 2048, 24, 2, 8, 8)
    n = len(lay)
    cross = sum(1 for a, d in enumerate(lay) for b in d["nb"] if a % 8 != b % 8)
    total = sum(len(d["nb"]) for d in lay)
    assert cross < 0.35 * total
    # a plain row-major deal would put almost every neighbour on another XCD
    assert total > 0 and n > 8


def test_no_layout_when_ring_too_deep():
    assert dtb.test_layout(4096, 4096, 8, 2, 8, 40) is None


# ----------------------------------------------------------------------------- tile-serial sweep

def _rects_tile(rects, region):
    """Rectangles [r0, r1) x [c0, c1) pairwise disjoint and covering `region` exactly."""
    area = sum((r1 - r0) * (c1 - c0) for r0, r1, c0, c1 in rects)
    R0, R1, C0, C1 = region
    assert area == (R1 - R0) * (C1 - C0)
    for r0, r1, c0, c1 in rects:
        assert R0 <= r0 < r1 <= R1 and C0 <= c0 < c1 <= C1
    for i in range(len(rects)):
        a = rects[i]
        for b in rects[i + 1:]:
            assert not (a[0] < b[1] and b[0] < a[1] and a[2] < b[3] and b[2] < a[3]), (a, b)


@pytest.mark.parametrize("case", [
    # rows, cols, R, C, waves, k, D, max_wg
    (600, 700, 8, 2, 8, 4, 16, 8),
    (1000, 333, 8, 2, 8, 3, 10, 6),
    (2048, 2048, 24, 2, 8, 8, 48, 64),
    (8192, 8192, 24, 2, 8, 8, 64, 256),
    (16384, 16384, 28, 4, 8, 8, 64, 256),
    (300, 5000, 16, 4, 8, 6, 20, 12),
], ids=lambda c: "x".join(map(str, c)))
def test_sweep_plan_properties(case):
    rows, cols, R, C, waves, k, D, max_wg = case
    ER, EC = waves * R, 64 * C
    tiles = dtb.test_sweep(rows, cols, R, C, waves, k, D, max_wg, 8)
    assert tiles is not None and len(tiles) >= 1
    valid = []
    for slots in tiles:
        nwg = slots[0]["nwg"]
        assert len(slots) == nwg <= max_wg
        st, cr = slots[0]["st"], slots[0]["cr"]
        # the computed region is the valid part grown by D, clipped to the interior
        assert cr == (max(st[0] - D, 1), min(st[1] + D, rows + 1), max(st[2] - D, 1), min(st[3] + D, cols + 1))
        valid.append(st)
        act = [(i, d) for i, d in enumerate(slots) if d["own_r0"] < d["own_r1"]]
        owned = [(d["own_r0"], d["own_r1"], d["own_c0"], d["own_c1"]) for _, d in act]
        _rects_tile(owned, cr)
        for i, d in act:
            f = (max(d["own_r0"] - k, cr[0]), min(d["own_r1"] + k, cr[1]),
                 max(d["own_c0"] - k, cr[2]), min(d["own_c1"] + k, cr[3]))
            assert d["ext_r0"] <= f[0] and f[1] <= d["ext_r0"] + ER
            assert d["ext_c0"] <= f[2] and f[3] <= d["ext_c0"] + EC
            assert 1 <= d["ext_r0"] and (rows < ER or d["ext_r0"] + ER - 1 <= rows)
            assert 1 <= d["ext_c0"] and (cols < EC or d["ext_c0"] + EC - 1 <= cols)
            want = sorted(j for j, o in act if j != i and o["own_r0"] < f[1] and o["own_r1"] > f[0]
                          and o["own_c0"] < f[3] and o["own_c1"] > f[2])
            assert sorted(d["nb"]) == want
    # valid parts partition the interior: every cell written exactly once per round
    _rects_tile(valid, (1, rows + 1, 1, cols + 1))


# ----------------------------------------------------------------------------- batched launch

def _check_batch(shapes, n_slots=256, r64=16, r32=16):
    res = dtb.test_batch(shapes, r64, r32, n_slots)
    assert res is not None
    jobs, lists = res
    assert sorted(j["prob"] for j in jobs) == list(range(len(shapes)))
    flags = set()
    members = {j: [] for j in range(len(jobs))}
    for s, lst in enumerate(lists):
        order = [job for job, _ in lst]
        assert order == sorted(order) and len(set(order)) == len(order), "slot work list not in global order"
        for job, local in lst:
            members[job].append(local)
    for j, J in enumerate(jobs):
        assert 1 <= J["g"] <= n_slots
        assert sorted(members[j]) == list(range(J["g"]))
        rng = set(range(J["flag_base"], J["flag_base"] + J["g"]))
        assert not (rng & flags)
        flags |= rng
        if j:
            assert jobs[j - 1]["start"] <= J["start"]
    # The batch's bounded waits outlast the longest legitimate wait: a member can wait at its job's
    # first synchronisation point for as long as the latest modelled start, and inside a job for
    # at most the job's duration; at 27 ns per poll (one s_sleep) the limit covers 8x the makespan.
    info = dtb.test_batch.last_info
    makespan = max(J["start"] + J["dur"] for J in jobs)
    assert abs(info["makespan_us"] - makespan) <= 2
    longest_wait_us = max(J["start"] for J in jobs) + max(J["dur"] for J in jobs)
    assert info["spin_limit"] >= 1 << 22
    assert info["spin_limit"] * 0.027 >= min(4 * longest_wait_us, 4e9 * 0.027)
    return jobs


def test_batch_plan_config5():
    from paper_2306_03336_amd import inputs
    probs = inputs.batched_set(5)
    jobs = _check_batch([(p.side, p.side, 0 if p.dtype == "f64" else 1, p.T) for p in probs])
    assert any(j["sweep"] for j in jobs) or max(p.side for p in probs) < 1700


def test_batch_plan_mixed_sizes():
    shapes = [(1, 1, 0, 5), (3000, 3000, 0, 100), (50, 2000, 1, 7), (4000, 100, 1, 300), (130, 130, 0, 0),
              (2100, 2100, 0, 30)]
    jobs = _check_batch(shapes)
    by_prob = {j["prob"]: j for j in jobs}
    assert by_prob[0]["g"] == 1 and not by_prob[0]["sweep"]
    assert by_prob[1]["sweep"] and by_prob[1]["ntiles"] >= 2
    assert by_prob[5]["sweep"]


def test_batch_plan_few_slots():
    jobs = _check_batch([(300, 300, 0, 10), (300, 300, 1, 10), (1000, 1000, 0, 20)], n_slots=4)
    assert max(j["g"] for j in jobs) <= 4


def test_batch_spin_limit_grows_with_makespan():
    """A batch with one long job: the wait bound follows the modelled makespan, not a fixed poll count."""
    short = _check_batch([(300, 300, 0, 10)])
    assert dtb.test_batch.last_info["spin_limit"] == 1 << 22
    _check_batch([(3000, 3000, 0, 200000), (200, 200, 1, 10), (500, 500, 0, 100)])
    info = dtb.test_batch.last_info
    assert info["makespan_us"] > 1e5
    assert info["spin_limit"] > 1 << 22
    assert info["spin_limit"] * 0.027 >= 8 * info["makespan_us"] * 0.999
    assert short


def test_batch_autotuner_picks_per_grid():
    """With the batched kernel's own instances (two tile shapes per precision), the planner chooses the tile
    shape, the exchange depth and (for grids larger than the chip) the round depth per grid: the 64-grid
    set ends up with both shapes of each precision and several k, and every choice is a candidate."""
    from paper_2306_03336_amd import inputs
    probs = inputs.batched_set(5)
    shapes = [(p.side, p.side, 0 if p.dtype == "f64" else 1, p.T) for p in probs]
    jobs = _check_batch(shapes, r64=0, r32=0)
    insts = {0: {(16, 2), (8, 4)}, 1: {(16, 4), (8, 4)}}
    used = {0: set(), 1: set()}
    for J in jobs:
        dt = shapes[J["prob"]][2]
        assert (J["R"], J["C"]) in insts[dt]
        used[dt].add((J["R"], J["C"]))
        assert 1 <= J["k"] <= 16
        if J["sweep"]:
            assert J["D"] in (16, 24, 32, 48, 64, 96, 128) and J["ntiles"] >= 1
    assert len({J["k"] for J in jobs}) >= 3
    assert used[0] == insts[0], used   # both FP64 shapes are in use
    # With slots to spare the planner takes the shortest candidate (a short, wide FP64 grid on 128 x 128
    # tiles at k = 16: 31 workgroups); with 24 slots the 64 x 256 tile's 14 workgroups win.
    jobs = _check_batch([(60, 3000, 0, 500), (700, 700, 0, 300)], r64=0, r32=0)
    assert (jobs[0]["R"], jobs[0]["C"], jobs[0]["g"], jobs[0]["k"]) == (16, 2, 31, 16)
    jobs = _check_batch([(60, 3000, 0, 500)], n_slots=24, r64=0, r32=0)
    assert (jobs[0]["R"], jobs[0]["C"]) == (8, 4) and jobs[0]["g"] <= 24


@pytest.mark.parametrize("n,E,K", [(1, 32, 3), (5, 32, 3), (31, 32, 3), (32, 32, 3), (33, 32, 3), (100, 32, 3),
                                   (512, 32, 3), (512, 128, 3), (513, 128, 2), (1000, 256, 1), (7, 7, 3), (64, 7, 3)])
def test_split3_covers_axis_with_deep_enough_rings(n, E, K):
    """The 3-D streaming split: owned parts tile 1 .. n exactly, in order; each range holds its owned part; an
    owned part keeps K cells from every open edge of its range (an edge at the storage ends 0 / n+1 is closed:
    the range holds the halo there)."""
    spans = dtb.test_split3(n, E, K)
    assert spans, (n, E, K)
    assert spans[0][1] == 1 and spans[-1][2] == n + 1
    for (e0, o0, o1), nxt in zip(spans, spans[1:] + [None]):
        assert o0 < o1 and e0 >= 0
        if nxt is not None:
            assert nxt[1] == o1
        lo_open = e0 > 0              # cells below the range exist (not the halo row 0 inside it)
        hi_open = e0 + E < n + 2      # the range ends before the far halo row n + 1
        assert o0 - e0 >= (K if lo_open else 1)
        assert e0 + E - o1 >= (K if hi_open else 0)


def test_zblock_choice_matches_the_measured_optima():
    """The z-block heights the 3-D planner picks at 512^3, where the alternatives were timed on an MI355X: FP64
    (bound by its memory traffic) keeps at least four workgroups per compute unit and, among those, the
    shortest modelled tail (51 planes: 11 blocks x 100 tiles, the last block 2 planes; 729 GCells/s against 681
    for 46 and 634-645 for 64-128); FP32 (compute-bound) takes deep blocks in whole waves of workgroups (128
    planes: one wave of 240 workgroups; with 4 columns per lane 905 against 893 for 64 and 801 for 18, with 3
    columns per lane, the instance the planner takes at this width, 1180 against 1181 for 64 and 951-988 for
    86-171)."""
    cells = 512 ** 3
    z64 = dtb.test_zblock(100, 32, 128, 3, 8, 512, cells)
    z32 = dtb.test_zblock(60, 32, 256, 3, 4, 512, cells)
    z32c3 = dtb.test_zblock(60, 32, 192, 3, 4, 512, cells)
    assert z64 == 51 and 100 * -(-512 // z64) >= 4 * 256
    assert z32 == 128 and z32c3 == 128
    # Shallow grids: a height within the grid; invalid arguments are refused.
    for depth in (1, 5, 30):
        z = dtb.test_zblock(100, 32, 128, 3, 8, depth, depth * 500 * 500)
        assert 1 <= z <= depth
    assert dtb.test_zblock(0, 32, 128, 3, 8, 512, cells) is None
    assert dtb.test_zblock(100, 32, 128, 3, 2, 512, cells) is None


def test_cols3_choice_takes_the_fewest_computed_columns():
    """FP32 has two streaming instances, 4 and 3 columns per lane (tiles 256 and 192 wide, K-deep rings on
    both sides); the planner takes the one whose overlapping spans compute fewer columns, 4 on a tie.  512
    columns: three spans of 256 (768 computed) against three of 192 (576): 3 (measured at 512^3, K = 3: 1180
    against 904 GCells/s, the same output bit for bit).  1000 columns: four of 256 (1024) against six of 192
    (1152): 4.  FP64 has one instance, 2."""
    def computed(n, c, K):
        return len(dtb.test_split3(n, 64 * c, K)) * 64 * c

    assert dtb.test_cols3(dtb.F32, 512, 3) == 3
    assert dtb.test_cols3(dtb.F32, 1000, 3) == 4
    assert dtb.test_cols3(dtb.F32, 250, 3) == 4     # one span of 256 against two of 192
    assert dtb.test_cols3(dtb.F32, 186, 3) == 3     # one span of each: 192 computed against 256
    for n in (1, 7, 100, 186, 187, 250, 251, 500, 512, 700, 1000, 1500, 4096):
        for K in (1, 2, 3):
            c = dtb.test_cols3(dtb.F32, n, K)
            assert computed(n, c, K) == min(computed(n, 4, K), computed(n, 3, K)), (n, K)
            if computed(n, 4, K) == computed(n, 3, K):
                assert c == 4, (n, K)
            assert dtb.test_cols3(dtb.F64, n, K) == 2
    assert dtb.test_cols3(dtb.F32, 0, 3) is None
    assert dtb.test_cols3(dtb.F32, 512, 4) is None
    assert dtb.test_cols3(2, 512, 3) is None


def test_split3_refuses_short_ranges():
    assert dtb.test_split3(100, 6, 3) is None     # E < 2K + 1
    assert dtb.test_split3(0, 32, 3) is None
