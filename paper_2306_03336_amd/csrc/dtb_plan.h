// dtb_plan.h -- the tile planner (host C++, no HIP calls; testable on a CPU).
//
// The whole-GPU tiling of the paper (Abstract, Section 1): a region of the
// grid is cut into one tile per workgroup such that all tiles together
// occupy the on-chip storage of the whole device, and every tile carries a
// ghost ring deep enough for k time steps between exchanges (Section 3.2).
// Grids larger than the chip are cut into big tiles processed one after
// another, several steps each (Section 3.3, Figure 1): the tile-serial sweep.
#pragma once
#include <stdint.h>

#include <vector>

#include "dtb_internal.h"

namespace dtb {

// Storage-coordinate rectangle [r0, r1) x [c0, c1).
struct Region {
    int r0 = 0, r1 = 0, c0 = 0, c1 = 0;
};

// Owned extents along one axis.  bounds has parts + 1 entries (storage
// coordinates, bounds[0] = lo, bounds[parts] = hi); ext0[i] is the storage
// coordinate of tile i's extended-tile origin.
struct AxisSplit {
    int parts = 0;
    std::vector<int> bounds;
    std::vector<int> ext0;
    bool narrow = false;  // the interior axis is shorter than the extended tile (the halo lies inside it)
};

// Split the range [lo, hi) of an interior axis of `dom` cells (storage
// coordinates 1..dom) into `parts` owned ranges whose k-deep fresh ring,
// clipped to [lo, hi), fits in an extended tile of `ext` cells placed inside
// the interior.  Returns false if that is impossible.
bool split_axis(int64_t lo, int64_t hi, int64_t dom, int ext, int k, int parts, AxisSplit* out);

// The same split written into caller-provided arrays (bounds: parts + 1
// entries, ext0: parts); allocates nothing.
bool split_axis_core(int64_t lo, int64_t hi, int64_t dom, int ext, int k, int parts, int* bounds, int* ext0,
                     bool* narrow);

// Smallest feasible number of parts (or 0 if none up to max_parts).
int min_parts(int64_t lo, int64_t hi, int64_t dom, int ext, int k, int max_parts);

// Lower bound on the parts an axis of len cells needs (0: none can hold it).
int first_parts_guess(int64_t len, int ext, int k);

// Launch slot of every tile of a pr x pc tile grid covering the region cr:
// the tile grid is cut into gy x gx blocks (gy * gx = n_xcd, blocks as square
// as possible in cells), the tiles are listed block by block (row-major inside
// a block), and the launch slots XCD by XCD (workgroup b runs on XCD
// (wg_base + b) % n_xcd) receive them in that order.  slot_of_tile and
// scratch: pr * pc entries each; allocates nothing.
void xcd_slot_order(int pr, int pc, const Region& cr, int n_xcd, int wg_base, int* slot_of_tile, int* scratch);

// Largest range one axis of `parts` tiles can cover.
int64_t axis_capacity(int ext, int k, int parts);

struct Layout {
    int R = 0, C = 0, waves = 0, ER = 0, EC = 0, k = 0;
    AxisSplit rows, cols;
    int nwg = 0;
    std::vector<WgDesc> wgs;  // indexed by blockIdx - wg_base
};

// Build the descriptor table for the computed region `cr` of a rows x cols
// interior (cells written back: `st`): tiles in an order that keeps each
// group of spatially adjacent tiles on one XCD ((wg_base + blockIdx) %
// n_xcd), and for every tile the list of tiles within k of it.  wg_base
// offsets every workgroup index (several problems in one launch); prob is
// stored in each descriptor.  Returns false if no layout exists or a
// neighbour list overflows.  neighbours = false leaves the lists empty
// (layouts whose workgroups never wait for each other).  A layout of more
// than max_tiles tiles is not built (returns false).
bool build_layout(int64_t rows, int64_t cols, const Region& cr, const Region& st, int R, int C, int waves, int k,
                  int n_xcd, int wg_base, int prob, Layout* out, bool neighbours = true, int max_tiles = INT32_MAX);

// The whole interior as computed and stored region.
inline Region interior(int64_t rows, int64_t cols) { return Region{1, (int)rows + 1, 1, (int)cols + 1}; }

// Time model (microseconds), calibrated on MI355X with one workgroup per
// compute unit: one time step of an ER x EC register tile (pts: 5 for j2d5pt,
// 9 for the 3 x 3 box), and one exchange (publish, flag wait, ghost load) of
// such a tile, through the LDS staging area or lane by lane.
double tile_step_time_us(int ER, int EC, int elem_bytes, int pts = 5);
double exchange_time_us(int ER, int EC, int R, int C, int elem_bytes, bool staged);

// Model time of one step of a resident layout on n_cu compute units holding
// slots_per_cu workgroups each: the compute units with the most tiles run
// all their steps, and one exchange every k steps (the exchanges of
// co-resident tiles overlap).  Infinite if the layout does not fit.
double layout_cost(const Layout& L, int slots_per_cu, int n_cu, int elem_bytes, int pts = 5);
double layout_cost_of(int nwg, int R, int C, int ER, int EC, int k, int slots_per_cu, int n_cu, int elem_bytes,
                      int pts = 5);

// ---- resident layout without allocation (the allocation-free entry point)

constexpr int kFixedMaxParts = 32;   // tiles per axis
constexpr int kFixedMaxWg = 256;     // tiles in all

// The whole interior of a rows x cols grid cut into pr x pc register tiles
// (the layout build_layout makes for a resident grid), in fixed-size arrays.
struct FixedLayout {
    int R = 0, C = 0, waves = 0, ER = 0, EC = 0, k = 0;
    int pr = 0, pc = 0, nwg = 0;
    bool narrow_rows = false, narrow_cols = false;
    int rb[kFixedMaxParts + 1], re0[kFixedMaxParts];  // row bounds and extended-tile origins (storage coordinates)
    int cb[kFixedMaxParts + 1], ce0[kFixedMaxParts];  // column bounds and origins
    int slot_of_tile[kFixedMaxWg];                     // launch slot of tile tr * pc + tc
};

// Build it; false if no layout exists within the fixed limits or a tile
// would have more than kMaxNeighbours neighbours.  Allocates nothing.
bool build_fixed_layout(int64_t rows, int64_t cols, int R, int C, int waves, int k, int n_xcd, FixedLayout* out);

// ---- tile-serial sweep

struct SweepPlan {
    int R = 0, C = 0, waves = 0, ER = 0, EC = 0, k = 0, D = 0;
    int tiles_r = 0, tiles_c = 0;        // big tiles per axis
    std::vector<int> vr, vc;             // valid (stored) bounds of the big tiles, storage coordinates
    int nwg = 0;                         // workgroups of the launch (max over big tiles)
    std::vector<Layout> tiles;           // one layout per big tile, row-major
    std::vector<WgDesc> table;           // [tile][nwg], idle workgroups padded in
    double est_cost = 0;                 // model cost per time step (arbitrary units)
};

// Plan the sweep of a rows x cols interior with big tiles whose computed
// region (valid part + D ring) fits in max_wg workgroups of the given
// register-tile instance.  Returns false if none fits.
bool plan_sweep(int64_t rows, int64_t cols, int R, int C, int waves, int k, int D, int max_wg, int n_xcd,
                SweepPlan* out);

// ---- batched launch

struct BatchSpec {
    int64_t rows = 0, cols = 0, pitch = 0, T = 0;
    int dtype = 0;
};

struct BatchJob {
    int prob = 0;
    int inst = 0;              // index into the planner's instance list
    int R = 0, C = 0;
    bool sweep = false;
    int g = 0;                 // workgroups of the group
    int k = 0, D = 0, ntiles = 1, nrounds = 1;
    int flag_base = 0, table_off = 0;
    std::vector<int> slots;    // launch slot of each member
    double start = 0, dur = 0; // model time (us)
    bool narrow_cols = false, narrow_rows = false;
};

struct BatchPlan {
    std::vector<BatchJob> jobs;       // in global order (by start time)
    std::vector<WgDesc> table;        // all jobs' descriptors
    std::vector<int> wl_off;          // nslots + 1 offsets into wl
    std::vector<int> wl_job, wl_local;
    int nslots = 0, nflags = 0;
    double makespan = 0;              // model time (us)
};

// Model time (us) of one step of a register tile of ER x EC cells of which
// `active_rows` rows hold grid rows (rows outside the grid are skipped).
double tile_step_us(int ER, int EC, int elem_bytes, int active_rows);

// Plan a batch.  Every problem becomes a job on a group of workgroups, chosen
// per problem among the instances of its precision, every exchange depth k
// and (for a grid larger than nslots tiles) every tile-serial round depth D:
// held on chip if it fits nslots tiles, else swept through big tiles.  Of a
// problem's candidates the planner takes the one with the least slot time
// (workgroups x modelled duration) among those no longer than the batch's
// lower bound on the makespan (the larger of the least total slot time over
// nslots and the longest least duration), else the shortest.  The jobs are
// then list-scheduled longest first onto the nslots launch slots, and every
// slot gets its (job, member) work list in one global job order.  Returns
// false if a problem fits no layout.
bool plan_batch(const std::vector<BatchSpec>& probs, const std::vector<TileInst>& insts, int waves, int nslots,
                BatchPlan* out);

// Poll limit of the batched kernel's bounded waits.  Under the list schedule a
// member may legitimately wait at its job's first synchronisation point for
// the rest of an earlier job on another member's slot -- up to the whole
// modelled makespan.  A poll takes at least one s_sleep (64 clocks, 27 ns at
// 2.4 GHz); the limit covers 8 times the modelled makespan at that rate, and
// never less than `floor` polls.
inline uint32_t batch_spin_limit(double makespan_us, uint32_t floor)
{
    const double polls = makespan_us * 8.0 / 0.027;
    if (!(polls > floor)) return floor;
    return polls >= 4.0e9 ? 4000000000u : (uint32_t)polls;
}

// ---- 3-D streaming (j3d7pt): overlapped tiles of one axis

// One tile of an axis of `n` interior cells (storage 0 .. n+1): extended range
// [e0, e0 + E), owned [own0, own1).
struct Span3 {
    int e0 = 0, own0 = 0, own1 = 0;
};

// Cover the interior 1 .. n of an axis with extended ranges of E cells whose
// owned parts stay K cells away from every open edge (an edge at the grid's
// halo is closed: the first range starts at the halo, the last one ends at
// it).  Returns false if E is too short for a K-deep ring (E < 2K + 1).
bool split_axis3(int64_t n, int E, int K, std::vector<Span3>* out);

// Model time (us) of one K-step streaming launch over nwg workgroups (tiles x
// z-blocks of zb planes) of an ER x EC tile, one workgroup per compute unit,
// for a grid of `depth` planes and `interior_cells` cells.  *bytes_bound (if
// given): the launch is bound by its memory traffic rather than its compute.
double stream3_launch_us(int nwg, int n_cu, int ER, int EC, int zb, int K, int elem_bytes, int64_t depth,
                         int64_t interior_cells, bool* bytes_bound = nullptr);

// The z-block height (planes) of a j3d7pt streaming plan with the least
// modelled launch time, for ntiles column tiles of ER x EC cells, K steps per
// launch, a grid of `depth` planes and `interior_cells` cells, on n_cu compute
// units (stream3_launch_us; see its definition for the measured rule).
int choose_zblock(int64_t ntiles, int ER, int EC, int K, int elem_bytes, int64_t depth, int64_t interior_cells,
                  int n_cu);

// Exchange points run_epochs performs for a segment of `steps` steps.
inline int exchanges_per_segment(int64_t steps, int k)
{
    const int64_t n = (steps + k - 1) / k - 1;
    return n > 0 ? (int)n : 1;
}

}  // namespace dtb
