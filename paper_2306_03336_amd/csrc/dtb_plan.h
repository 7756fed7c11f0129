// dtb_plan.h -- the tile planner (host C++, no HIP calls; testable on a CPU).
//
// The whole-GPU tiling of the paper (Abstract, Section 1): the grid is cut
// into one tile per workgroup such that all tiles together occupy the
// on-chip storage of the whole device, and every tile carries a ghost ring
// deep enough for k time steps between exchanges (Section 3.2).
#pragma once
#include <stdint.h>

#include <vector>

#include "dtb_internal.h"

namespace dtb {

// Owned extents along one axis.  bounds has parts + 1 entries (storage
// coordinates, bounds[0] = 1, bounds[parts] = len + 1); ext0[i] is the storage
// coordinate of tile i's extended-tile origin.
struct AxisSplit {
    int parts = 0;
    std::vector<int> bounds;
    std::vector<int> ext0;
    bool narrow = false;  // the axis is shorter than the extended tile (halo lies inside it)
};

// Split an interior axis of `len` cells into `parts` owned ranges whose
// k-deep fresh ring fits in an extended tile of `ext` cells.  Returns false
// if that is impossible.
bool split_axis(int64_t len, int ext, int k, int parts, AxisSplit* out);

// Smallest feasible number of parts (or 0 if none up to max_parts).
int min_parts(int64_t len, int ext, int k, int max_parts);

struct Layout {
    int R = 0, C = 0, waves = 0, ER = 0, EC = 0, k = 0;
    AxisSplit rows, cols;
    int nwg = 0;
    std::vector<WgDesc> wgs;  // indexed by blockIdx
};

// Build the descriptor table for one problem: tiles in an order that keeps
// each group of spatially adjacent tiles on one XCD (blockIdx % n_xcd), and
// for every tile the list of tiles within k of it.  wg_base offsets every
// workgroup index (for packing several problems into one launch); prob is
// stored in each descriptor.  Returns false if a neighbour list overflows.
bool build_layout(int64_t rows, int64_t cols, int R, int C, int waves, int k, int n_xcd, int wg_base,
                  int prob, Layout* out);

// Static cost estimate of one step of a layout on a device with `slots`
// co-resident workgroup slots: cells each compute unit advances per step,
// times a factor for the exchange every k steps.
double layout_cost(const Layout& L, int slots_per_cu, int n_cu, double sync_steps);

}  // namespace dtb
