// dtb_internal.h -- descriptors shared by the host planner and the gfx950 kernels.
//
// Not part of the public C ABI (include/dtb.h).  Every field is plain data so
// the planner can build the tables on the host and copy them to the device
// once per plan.
#pragma once
#include <stdint.h>

namespace dtb {

constexpr int kWaveSize = 64;
constexpr int kMaxNeighbours = 24;

// Border strips go through the LDS staging area when the tile's two
// register sets leave room for the staging code (at most 192 VGPRs per lane)
// and the ring is at most stage_k(R) deep; otherwise lane by lane.  Shared by
// the kernels (which size the area) and the planner (which prices it).
constexpr int stage_k(int R) { return R >= 12 ? 12 : 8; }
constexpr bool tile_stages(int R, int C, int elem_bytes) { return 2 * R * C * elem_bytes / 4 <= 192; }
constexpr bool exchange_staged(int R, int C, int elem_bytes, int k)
{
    return tile_stages(R, C, elem_bytes) && k <= stage_k(R);
}

// Epoch flags live kFlagStride uint32 apart (4 KiB): every flag in its own
// cache line and, whatever the channel interleave, spread over the HBM
// channels, so polling workgroups do not queue on one channel.
constexpr int kFlagStride = 1024;

// Device-wide barrier counters of the tile-serial sweep (and of the
// grid-barrier design): slots kFlagStride apart, reset before every launch.
constexpr int kBarrierSlots = 18;

// One problem of a launch: a grid advanced T steps in place.
//
// Storage (same for grid and the two exchange buffers): (rows + 2) lines of
// `pitch` elements, row-major; interior rows 1..rows, columns 1..cols; the
// one-cell ring around it is the fixed Dirichlet halo.
struct ProbDesc {
    void* grid;          // caller's storage, updated in place
    void* xbuf[2];       // exchange buffers (same layout), owned by the plan
    int64_t pitch;       // elements per storage row
    int64_t T;           // time steps
    int32_t rows, cols;  // interior size
    int32_t k;           // steps between inter-workgroup halo exchanges
    int32_t wg0, nwg;    // this problem's workgroups: blockIdx-independent ids wg0..wg0+nwg-1
    int32_t dtype;       // 0 = FP64, 1 = FP32
    int32_t fma;         // 1: fused multiply-add chain; 0: separate products summed W,E,S,C,N
    int32_t narrow_cols; // 1 when some tile holds the east halo column inside it
    int32_t narrow_rows; // 1 when some tile holds the south halo row inside it
    int32_t debug;       // DTB_DEBUG_* bits (include/dtb.h)
    double coeffs[9];    // j2d5pt: c, n, s, e, w; j2d9pt: sw, s, se, w, c, e, nw, n, ne
    uint64_t* timing;    // DTB_DEBUG_TIMING: kTimingSlots counters per workgroup, else null
    int32_t direct_xchg; // 1: exchange border strips lane by lane, never through the LDS staging area
    int32_t grid_sync;   // 1: a device-wide barrier at every exchange point instead of neighbour flags
    uint32_t* bar;       // grid_sync: the barrier's counters (kBarrierSlots slots, reset before each launch)
};

// Per-workgroup phase timing (s_memrealtime ticks, 100 MHz): time in steps,
// in publishing border strips (stores and their completion), waiting for
// neighbours' flags, loading the ghost ring, and the number of exchanges.
constexpr int kTimingSlots = 11;
constexpr int kEpochTimingSlots = 8;  // the slots kept per thread through the epoch loop (registers)
// With the LDS staging area, publishing and loading are each split in two:
// kTimeStageOut (registers to LDS) + kTimePublish (LDS to the buffer), and
// kTimeStageIn (buffer to LDS) + kTimeGhost (LDS to registers).
// kTimeLoad / kTimeStore: loading the extended tile and storing the owned
// cells (once per segment); kTimeBarrier: the tile-serial sweep's device-wide
// barrier between big tiles.  These three lie outside kTimeTotal.
enum TimingSlot { kTimeSteps = 0, kTimePublish = 1, kTimeWait = 2, kTimeGhost = 3, kTimeExchanges = 4,
                  kTimeTotal = 5, kTimeStageOut = 6, kTimeStageIn = 7, kTimeLoad = 8, kTimeStore = 9,
                  kTimeBarrier = 10 };

// One workgroup: which problem, where its register tile sits, what it owns.
//
// The extended tile is ER x EC cells (ER = waves * rows per lane, EC = 64 *
// columns per lane); its cell (0, 0) is storage cell (ext_r0, ext_c0).  The
// owned cells are [own_r0, own_r1) x [own_c0, own_c1) in storage
// coordinates; the owned regions of the workgroups working on one region
// tile it exactly.  That region (the computed region, cr_*) is the whole
// interior for a grid held on chip, or one big tile plus its D-deep ring for
// the tile-serial sweep; ghost cells are only refreshed inside it.  Of the
// owned cells, those inside st_* are written back (the whole interior, or
// the big tile's valid part).  nb[] lists the workgroups (same numbering as
// the launch) whose owned cells lie within k of this one's, i.e. those it
// exchanges halos with.  An idle workgroup (no owned cells) has own_r0 ==
// own_r1.
struct alignas(16) WgDesc {
    int32_t prob;
    int32_t ext_r0, ext_c0;
    int32_t own_r0, own_r1, own_c0, own_c1;
    int32_t nnb;
    int32_t cr_r0, cr_r1, cr_c0, cr_c1;
    int32_t st_r0, st_r1, st_c0, st_c1;
    int32_t nb[kMaxNeighbours];
};

// One job of a batched launch: a problem run by a group of g workgroups,
// held on chip for all its steps (ntiles = nrounds = 1, D = T, in place) or
// swept through big tiles with `ws` as the second buffer.
struct JobDesc {
    int32_t prob;
    int32_t g;          // workgroups in the group
    int32_t flag_base;  // flags[flag_base + i] belong to group member i
    int32_t table_off;  // descriptors: table[table_off + tile * g + i]
    int32_t ntiles;
    int32_t D;
    int32_t nrounds;
    int32_t sweep;
    int32_t R, C;       // the register-tile instance: rows and columns per lane
    void* ws;
};

// A register-tile instance the batched kernel carries: precision (0 = FP64,
// 1 = FP32), rows and columns per lane (8 waves per workgroup).
struct TileInst {
    int dtype = 0, R = 0, C = 0;
};

// Entry of a launch slot's work list: job index and the slot's member index in it.
struct WorkItem {
    int32_t job, local;
};

// ---- j3d7pt streaming (dtb_stream3d.h)

constexpr int kStreamWaves = 8;

// One workgroup's work: an (x, y) tile and a block of planes.
struct Tile3Desc {
    int32_t ext_r0, ext_c0;   // storage row / column of the extended tile's first row / column (may be 0: halo)
    int32_t own_r0, own_r1;   // owned rows [own_r0, own_r1), storage coordinates
    int32_t own_c0, own_c1;   // owned columns
    int32_t edge;             // the extended tile holds cells outside the interior (halo or beyond the grid)
    int32_t pad_;
};

struct Stream3Args {
    const void* src;
    void* dst;
    int64_t pitch, plane_pitch;
    int32_t depth, rows, cols;
    int32_t zb;               // planes per z-block
    int32_t nzb;              // z-blocks
    int32_t ntiles;           // (x, y) tiles
    double coeffs[7];         // c, n, s, e, w, t, b
};

}  // namespace dtb
