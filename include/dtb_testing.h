/*
 * dtb_testing.h -- hooks into libdtb for tests and measurements: the planner
 * without a GPU, and micro-benchmarks of the part the kernels run on.  Not
 * needed to use the library.
 */
#ifndef LIBDTB_DTB_TESTING_H
#define LIBDTB_DTB_TESTING_H

#include <stdint.h>

#include "dtb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DTB_TEST_MAX_NEIGHBOURS 24
#define DTB_TEST_LAYOUT_STRIDE (8 + DTB_TEST_MAX_NEIGHBOURS)

/*
 * Run the resident-path tile planner for an interior of rows x cols with a
 * register tile of (waves * rows_per_lane) x (64 * cols_per_lane) cells and
 * exchange depth k, workgroups dealt over n_xcd XCDs.  No HIP call is made.
 *
 * Returns the number of workgroups (tiles), or -1 if no layout exists.  If
 * that number is <= max_wg, `out` (max_wg * DTB_TEST_LAYOUT_STRIDE int32,
 * caller-owned) receives one record per workgroup in launch order:
 *   ext_r0, ext_c0, own_r0, own_r1, own_c0, own_c1, n_neighbours,
 *   neighbours[DTB_TEST_MAX_NEIGHBOURS] (-1 padded), flags
 * where coordinates are storage coordinates (the halo is row/column 0),
 * owned ranges are half-open, and flags bit 0 / bit 1 mark an axis shorter
 * than the register tile (rows / columns).
 */
int32_t dtb_test_layout(int64_t rows, int64_t cols, int32_t rows_per_lane, int32_t cols_per_lane, int32_t waves,
                        int32_t k, int32_t n_xcd, int32_t* out, int32_t max_wg);

#define DTB_TEST_SWEEP_STRIDE (17 + DTB_TEST_MAX_NEIGHBOURS)

/*
 * Run the tile-serial sweep planner (big tiles of depth D over an interior of
 * rows x cols, at most max_wg workgroups per big tile).  No HIP call is made.
 *
 * Returns the number of records (big tiles x workgroups of the launch), or -1
 * if no plan exists.  If that number is <= max_records, `out` (max_records *
 * DTB_TEST_SWEEP_STRIDE int32, caller-owned) receives, per big tile and
 * launch slot: tile index, workgroups of the launch, ext_r0, ext_c0, own_r0,
 * own_r1, own_c0, own_c1, computed region (r0, r1, c0, c1), stored region
 * (r0, r1, c0, c1), n_neighbours, neighbours[DTB_TEST_MAX_NEIGHBOURS].  An
 * idle slot has own_r0 == own_r1.
 */
int32_t dtb_test_sweep(int64_t rows, int64_t cols, int32_t rows_per_lane, int32_t cols_per_lane, int32_t waves,
                       int32_t k, int32_t D, int32_t max_wg, int32_t n_xcd, int32_t* out, int32_t max_records);

/*
 * The 3-D streaming planner's split of one axis of n interior cells (storage
 * 0 .. n+1) into overlapping ranges of E cells with K-deep rings at open
 * edges (dtb_plan3d): writes up to max_spans triples (e0, own0, own1) -- the
 * range [e0, e0 + E) and its owned part [own0, own1) -- and returns the number
 * of ranges (more than max_spans: nothing written), or -1 if E < 2K + 1 or an
 * argument is invalid.  Host only.
 */
int32_t dtb_test_split3(int64_t n, int32_t E, int32_t K, int32_t* out, int32_t max_spans);

/*
 * The z-block height (planes per block) the j3d7pt planner (dtb_plan3d)
 * picks when the caller leaves it open, for ntiles column tiles of
 * ext_rows x ext_cols cells, K steps per launch, elem_bytes 8 (FP64) or 4
 * (FP32), a grid of `depth` planes and `interior_cells` interior cells, on
 * n_cu compute units.  Returns -1 if an argument is invalid.  Host only.
 */
int32_t dtb_test_zblock(int64_t ntiles, int32_t ext_rows, int32_t ext_cols, int32_t K, int32_t elem_bytes,
                        int64_t depth, int64_t interior_cells, int32_t n_cu);

/*
 * The columns per lane of the streaming instance the j3d7pt planner
 * (dtb_plan3d) picks when cols_per_lane is left open, for a grid `cols`
 * interior columns wide, dtype DTB_F64 or DTB_F32 and K steps per launch
 * (1 .. 3).  Returns -1 if an argument is invalid.  Host only.
 */
int32_t dtb_test_cols3(int32_t dtype, int64_t cols, int32_t K);

#define DTB_TEST_BATCH_STRIDE 13

/*
 * Run the batch planner for `count` problems (rows[i] x cols[i], dtype[i],
 * T[i]) on n_slots workgroup slots.  r64 = r32 = 0: with the register-tile
 * instances the batched kernel carries; otherwise with one instance per
 * precision, FP64 2 x r64 and FP32 4 x r32 cells per lane.  No HIP call is
 * made.  Returns the number of jobs (== count), or -1.
 * `jobs` (count * DTB_TEST_BATCH_STRIDE int32, may be NULL) receives, in
 * global job order: problem, workgroups, sweep (0/1), ntiles, D, nrounds,
 * flag_base, table_off, start (model us, rounded), duration (model us),
 * exchange depth k, rows per lane, columns per lane.
 * `slot_lists` (may be NULL; n_slots + 1 offsets followed by the
 * (job, member) pairs, 2 int32 each; size n_slots + 1 + 2 * total members)
 * receives every slot's work list.  `info` (may be NULL, 2 int64) receives the
 * modelled makespan (us) and the poll limit of the batch's bounded waits.
 */
int32_t dtb_test_batch(int32_t count, const int64_t* rows, const int64_t* cols, const int32_t* dtype,
                       const int64_t* T, int32_t r64, int32_t r32, int32_t n_slots, int32_t* jobs,
                       int32_t* slot_lists, int32_t slot_lists_len, int64_t* info);

/* Micro-benchmark kinds for dtb_probe. */
#define DTB_PROBE_LDS_READ 0  /* LDS reads, 16 bytes per lane, conflict-free; nwg workgroups (0: 2 per CU) */
#define DTB_PROBE_LDS_WRITE 1 /* LDS writes, likewise */
#define DTB_PROBE_COPY 2      /* device-to-device copy of `size` bytes, `iters` times, 16 bytes per lane */
#define DTB_PROBE_BARRIER 3   /* `iters` device-wide barriers among nwg persistent workgroups (0: one per CU) */
#define DTB_PROBE_FLAGS 4     /* `iters` neighbour exchange points (flag raised, 8 neighbours awaited), no data */

/*
 * Run one micro-benchmark on the current device, enqueued on `stream` (a
 * hipStream_t as void*, NULL = default stream) and timed there with HIP events;
 * waits for it.  out[0] receives the elapsed milliseconds of the timed part and
 * out[1] the work it did: bytes moved (LDS, copy: read + written) or the
 * number of barriers / exchange points.  Allocates and frees its own buffers
 * (not for use under stream capture).  DTB_ERR_NOT_CORESIDENT if a persistent
 * probe asks for more workgroups than compute units; DTB_ERR_TIMEOUT if a
 * bounded wait expired.
 */
dtb_status dtb_probe(int32_t kind, int64_t size, int32_t iters, int32_t nwg, void* stream, double* out);

#ifdef __cplusplus
}
#endif

#endif /* LIBDTB_DTB_TESTING_H */
