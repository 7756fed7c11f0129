// dtb_launch.h -- host-side entry points into the kernels of dtb_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtb_internal.h"

namespace dtb {

// One step of the untiled baseline; pts 5: j2d5pt (five coefficients c, n, s,
// e, w), 9: the 3 x 3 box (nine, sw .. ne).
hipError_t launch_step(int dtype, bool fma, const void* in, void* out, int64_t pitch, int rows, int cols,
                       const double* coeffs, hipStream_t st, int pts = 5);
hipError_t launch_copy_interior(int dtype, const void* src, void* dst, int64_t pitch, int rows, int cols,
                                hipStream_t st);
hipError_t launch_copy_halo(int dtype, const void* src, void* dst, int64_t pitch, int rows, int cols,
                            hipStream_t st);

// The DTB kernel for (dtype, rows per lane R, variant, stencil), or nullptr
// when that R is not instantiated.  *C receives the columns per lane and
// *waves the waves per workgroup of the instance.  want_waves: 0 or 8 for the
// standard 8-wave workgroups, 4 for the half-height instances (FP64 R = 24
// only).  pts: 5 (j2d5pt) or 9 (the 3 x 3 box: FP64 R = 8, FP32 R = 16, both
// with 4 columns per lane).
const void* dtb_kernel(int dtype, int R, bool fma, bool colmask, bool rowcheck, int* C, int* waves,
                       int want_waves = 0, int pts = 5);

// The tile-serial sweep kernel of the same instance (arguments: ProbDesc,
// SweepArgs, descriptor table, flags, error word, spin limit).
const void* dtb_sweep_kernel(int dtype, int R, bool fma, bool colmask, bool rowcheck, int* C, int* waves,
                             int pts = 5);

// Arguments of the sweep kernel besides the problem.
struct SweepArgs {
    void* bufs[2];   // round r reads bufs[r & 1], writes bufs[(r + 1) & 1]; bufs[0] is the grid
    int32_t ntiles, nwg, D, nrounds;
    uint32_t* bar;   // device-wide barrier counters: 17 slots kFlagStride apart (reset before every launch)
};

hipError_t launch_reset_counter(uint32_t* bar, hipStream_t st);

// The overlapped per-workgroup blocking kernel of the same instance
// (arguments: ProbDesc, descriptor table, source buffer, destination buffer,
// steps), or nullptr where it is not instantiated (FP64 2 x 8, 2 x 24, 4 x 12;
// FP32 4 x 8, 4 x 24).
const void* dtb_ovl_kernel(int dtype, int R, bool fma, bool colmask, bool rowcheck, int* C, int* waves);

// ---- j3d7pt (dtb_inst_3d.hip)

// The K-step streaming kernel (arguments: Stream3Args, Tile3Desc table) for
// dtype, K (1 .. 3) and columns per lane (0: the default instance), or
// nullptr; *C, *R: columns and rows per lane.
const void* dtb_stream3d_kernel(int dtype, int K, bool fma, int cols_per_lane, int* C, int* R);
// One step of the untiled baseline (seven coefficients c, n, s, e, w, t, b).
hipError_t launch_step3d(int dtype, bool fma, const void* in, void* out, int64_t pitch, int64_t plane_pitch,
                         int depth, int rows, int cols, const double* coeffs, hipStream_t st);
hipError_t launch_copy_shell3d(int dtype, const void* src, void* dst, int64_t pitch, int64_t plane_pitch, int depth,
                               int rows, int cols, hipStream_t st);
hipError_t launch_copy_interior3d(int dtype, const void* src, void* dst, int64_t pitch, int64_t plane_pitch,
                                  int depth, int rows, int cols, hipStream_t st);

// The batched persistent kernel (arguments: ProbDesc*, JobDesc*, WgDesc*
// table, work-list offsets, work items, flags, error word, spin limit); the
// register-tile instances it carries (at most kMaxBatchInsts) into insts,
// their number into *n.
constexpr int kMaxBatchInsts = 8;
const void* batched_kernel(TileInst* insts, int* n);

}  // namespace dtb
