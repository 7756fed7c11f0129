/*
 * dtb_testing.h -- host-only hooks into libdtb's planner, for tests that run
 * without a GPU.  Not needed to use the library.
 */
#ifndef LIBDTB_DTB_TESTING_H
#define LIBDTB_DTB_TESTING_H

#include <stdint.h>

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

#define DTB_TEST_BATCH_STRIDE 10

/*
 * Run the batch planner for `count` problems (rows[i] x cols[i], dtype[i],
 * T[i]) on n_slots workgroup slots with register tiles of r64 / r32 rows per
 * lane.  No HIP call is made.  Returns the number of jobs (== count), or -1.
 * `jobs` (count * DTB_TEST_BATCH_STRIDE int32, may be NULL) receives, in
 * global job order: problem, workgroups, sweep (0/1), ntiles, D, nrounds,
 * flag_base, table_off, start (model us, rounded), duration (model us).
 * `slot_lists` (may be NULL; n_slots + 1 offsets followed by the
 * (job, member) pairs, 2 int32 each; size n_slots + 1 + 2 * total members)
 * receives every slot's work list.
 */
int32_t dtb_test_batch(int32_t count, const int64_t* rows, const int64_t* cols, const int32_t* dtype,
                       const int64_t* T, int32_t r64, int32_t r32, int32_t n_slots, int32_t* jobs,
                       int32_t* slot_lists, int32_t slot_lists_len);

#ifdef __cplusplus
}
#endif

#endif /* LIBDTB_DTB_TESTING_H */
