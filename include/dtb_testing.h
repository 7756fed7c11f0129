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

#ifdef __cplusplus
}
#endif

#endif /* LIBDTB_DTB_TESTING_H */
