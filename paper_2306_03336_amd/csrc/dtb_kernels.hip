// dtb_kernels.hip -- gfx950 kernels for the j2d5pt iterative stencil (and the
// one-step baseline of the 3 x 3 box, j2d9pt).
//
// The update (Listing 1 of Zhang et al., GPGPU '23): every interior cell
// becomes w*W + e*E + s*S + c*C + n*N of the previous step's values, with
// W = (i, j-1), E = (i, j+1), S = (i-1, j), N = (i+1, j) (x = column j is the
// contiguous index, y = row i).  Reads and writes never alias within a step
// (Jacobi).  The one-cell ring around the interior is a fixed Dirichlet halo.
//
// This file holds the untiled baseline and the host-side launchers; the
// deep-temporal-blocking kernels are templates in dtb_tile.h, instantiated in
// dtb_inst_*.hip.
//
//  * k_step: one time step per launch, global memory to global memory.  It is
//    the untiled baseline the paper starts from before the time loop moves
//    into the kernel (Section 3.1).  Bound by HBM (or the Infinity Cache when
//    the two buffers fit in it): one read and one write per cell-update.
//
//  * k_dtb: deep temporal blocking (Sections 1, 3.1-3.3, Figure 1).  One
//    persistent cooperative launch runs every time step.  Each workgroup keeps
//    an extended tile -- its owned cells plus a ghost ring k cells deep -- in
//    the VGPR file (two register sets, ping-ponged between steps), advances it
//    k steps without touching HBM, then exchanges the k-deep border strips with
//    the workgroups around it through global memory and per-workgroup epoch
//    flags (bulk-synchronous, Section 3.2; a neighbour-wise form of the grid
//    barrier).  Inside a workgroup the waves are stacked vertically; each step
//    they swap their top and bottom rows through LDS and meet at one s_barrier.
//    East/west neighbours across lanes come from DPP wave shifts.
//
// Arithmetic: with fma == 0 every product is rounded and the sum is taken
// left to right in the order W, E, S, C, N (the printed order of Listing 1);
// with fma == 1 the same chain uses fused multiply-adds.  The library is built
// with -ffp-contract=off so the compiler never fuses on its own.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dtb_internal.h"
#include "dtb_launch.h"
#include "dtb_stencil.h"

namespace dtb {

// ============================================================================ one-step baseline

// Block: 64 x 4 threads.  Thread (tx, ty) owns column j and STEP_ILP
// consecutive rows; it keeps the column's vertical neighbours in registers
// (the column cache of Listing 1) and reads W/E from memory (cache hits).
constexpr int kStepIlp = 8;

template <typename T, bool FMA>
__global__ __launch_bounds__(256) void k_step(const T* __restrict__ in, T* __restrict__ out,
                                              int64_t pitch, int rows, int cols,
                                              Coef<T> k)
{
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i0 = (blockIdx.y * 4 + threadIdx.y) * kStepIlp + 1;
    if (j > cols || i0 > rows) return;
    T col[kStepIlp + 2];
#pragma unroll
    for (int q = 0; q < kStepIlp + 2; ++q) {
        const int i = i0 - 1 + q;
        col[q] = (i <= rows + 1) ? in[(int64_t)i * pitch + j] : T(0);
    }
#pragma unroll
    for (int q = 0; q < kStepIlp; ++q) {
        const int i = i0 + q;
        if (i <= rows) {
            const T* mid = in + (int64_t)i * pitch;
            out[(int64_t)i * pitch + j] = j2d5pt<FMA>(mid[j - 1], mid[j + 1], col[q], col[q + 1], col[q + 2], k);
        }
    }
}

// The same step with one 16-byte access per lane: lane l of a wave holds the V
// = 16 / sizeof(T) consecutive columns starting at storage column
// (64 * blockIdx.x + l) * V (2 FP64 or 4 FP32 values), for kStepRows rows plus
// the row above and below (the column cache of Listing 1, V columns wide).
// West/east neighbours of a lane's first and last column come from the
// neighbouring lanes by DPP wave shifts; lanes 0 and 63 read theirs from
// memory.  Needs rows that start 16-byte aligned (16-byte aligned base, pitch a
// multiple of V); the launcher falls back to k_step otherwise.  Same operands,
// same order of operations as k_step: bit for bit the same result.
constexpr int kStepRows = 8;

template <typename T>
__device__ __forceinline__ T lane_shr1(T v)  // lane l gets lane l-1's value (lane 0: 0)
{
    return __builtin_amdgcn_update_dpp((T)0, v, 0x138, 0xf, 0xf, true);
}
template <typename T>
__device__ __forceinline__ T lane_shl1(T v)  // lane l gets lane l+1's value (lane 63: 0)
{
    return __builtin_amdgcn_update_dpp((T)0, v, 0x130, 0xf, 0xf, true);
}

template <typename T, bool FMA>
__global__ __launch_bounds__(256) void k_step_vec(const T* __restrict__ in, T* __restrict__ out, int64_t pitch,
                                                  int rows, int cols, Coef<T> k)
{
    constexpr int V = 16 / (int)sizeof(T);
    using VT = std::conditional_t<sizeof(T) == 8, double2, float4>;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int j0 = (blockIdx.x * 64 + lane) * V;  // storage column of this lane's first value
    const int i0 = (blockIdx.y * 4 + wave) * kStepRows + 1;
    if (i0 > rows) return;  // the whole wave
    const bool inrow = j0 <= cols + 1;  // this lane's group lies in the row's storage (pitch is a multiple of V)
    T c[kStepRows + 2][V];
#pragma unroll
    for (int q = 0; q < kStepRows + 2; ++q) {
        const int i = i0 - 1 + q;
        VT v{};
        if (inrow && i <= rows + 1) v = *(const VT*)(in + (int64_t)i * pitch + j0);
        const T* e = (const T*)&v;
#pragma unroll
        for (int x = 0; x < V; ++x) c[q][x] = e[x];
    }
#pragma unroll
    for (int q = 0; q < kStepRows; ++q) {
        const int i = i0 + q;
        if (i > rows) break;  // uniform: the wave's rows
        const T* row = in + (int64_t)i * pitch;
        T wv = lane_shr1(c[q + 1][V - 1]);
        T ev = lane_shl1(c[q + 1][0]);
        if (lane == 0 && j0 >= 1 && inrow) wv = row[j0 - 1];
        if (lane == 63 && j0 + V <= cols + 1) ev = row[j0 + V];
        T r[V];
#pragma unroll
        for (int x = 0; x < V; ++x) {
            const T W = x == 0 ? wv : c[q + 1][x - 1];
            const T E = x == V - 1 ? ev : c[q + 1][x + 1];
            r[x] = j2d5pt<FMA>(W, E, c[q][x], c[q + 1][x], c[q + 2][x], k);
        }
        T* orow = out + (int64_t)i * pitch;
        if (j0 >= 1 && j0 + V - 1 <= cols) {
            VT v;
            T* e = (T*)&v;
#pragma unroll
            for (int x = 0; x < V; ++x) e[x] = r[x];
            *(VT*)(orow + j0) = v;
        } else if (inrow) {
#pragma unroll
            for (int x = 0; x < V; ++x)
                if (j0 + x >= 1 && j0 + x <= cols) orow[j0 + x] = r[x];
        }
    }
}

// ---- the 3 x 3 box (j2d9pt): the same two one-step kernels.  Every output
// cell is the weighted sum of its 3 x 3 block of the previous step's values
// (weights in the order sw, s, se, w, c, e, nw, n, ne; S = row i-1), products
// summed in that order.

// Thread (tx, ty) owns column j and kStepIlp consecutive rows, and keeps the
// three columns j-1, j, j+1 of those rows and the rows above and below in
// registers.
template <typename T, bool FMA>
__global__ __launch_bounds__(256) void k_step9(const T* __restrict__ in, T* __restrict__ out, int64_t pitch,
                                               int rows, int cols, Coef9<T> k)
{
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i0 = (blockIdx.y * 4 + threadIdx.y) * kStepIlp + 1;
    if (j > cols || i0 > rows) return;
    T cw[kStepIlp + 2], cm[kStepIlp + 2], ce[kStepIlp + 2];
#pragma unroll
    for (int q = 0; q < kStepIlp + 2; ++q) {
        const int i = i0 - 1 + q;
        const T* row = in + (int64_t)i * pitch;
        const bool ok = i <= rows + 1;
        cw[q] = ok ? row[j - 1] : T(0);
        cm[q] = ok ? row[j] : T(0);
        ce[q] = ok ? row[j + 1] : T(0);
    }
#pragma unroll
    for (int q = 0; q < kStepIlp; ++q) {
        const int i = i0 + q;
        if (i <= rows) {
            const T a[9] = {cw[q], cm[q], ce[q], cw[q + 1], cm[q + 1], ce[q + 1], cw[q + 2], cm[q + 2], ce[q + 2]};
            out[(int64_t)i * pitch + j] = j2d9pt<FMA>(a, k);
        }
    }
}

// 16-byte groups as in k_step_vec; a lane's west/east neighbours in each of
// the three rows come from the neighbouring lanes (lanes 0 and 63 read theirs
// from memory).
template <typename T, bool FMA>
__global__ __launch_bounds__(256) void k_step9_vec(const T* __restrict__ in, T* __restrict__ out, int64_t pitch,
                                                   int rows, int cols, Coef9<T> k)
{
    constexpr int V = 16 / (int)sizeof(T);
    using VT = std::conditional_t<sizeof(T) == 8, double2, float4>;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int j0 = (blockIdx.x * 64 + lane) * V;
    const int i0 = (blockIdx.y * 4 + wave) * kStepRows + 1;
    if (i0 > rows) return;  // the whole wave
    const bool inrow = j0 <= cols + 1;
    // c[q][0] and c[q][V + 1]: the west and east neighbours of the group in row i0 - 1 + q.
    T c[kStepRows + 2][V + 2];
#pragma unroll
    for (int q = 0; q < kStepRows + 2; ++q) {
        const int i = i0 - 1 + q;
        const bool ok = inrow && i <= rows + 1;
        VT v{};
        if (ok) v = *(const VT*)(in + (int64_t)i * pitch + j0);
        const T* e = (const T*)&v;
#pragma unroll
        for (int x = 0; x < V; ++x) c[q][x + 1] = e[x];
        T wv = lane_shr1(c[q][V]);
        T ev = lane_shl1(c[q][1]);
        if (lane == 0 && j0 >= 1 && ok) wv = in[(int64_t)i * pitch + j0 - 1];
        if (lane == 63 && j0 + V <= cols + 1 && ok) ev = in[(int64_t)i * pitch + j0 + V];
        c[q][0] = wv;
        c[q][V + 1] = ev;
    }
#pragma unroll
    for (int q = 0; q < kStepRows; ++q) {
        const int i = i0 + q;
        if (i > rows) break;  // uniform: the wave's rows
        T r[V];
#pragma unroll
        for (int x = 0; x < V; ++x) {
            const T a[9] = {c[q][x], c[q][x + 1], c[q][x + 2], c[q + 1][x], c[q + 1][x + 1], c[q + 1][x + 2],
                            c[q + 2][x], c[q + 2][x + 1], c[q + 2][x + 2]};
            r[x] = j2d9pt<FMA>(a, k);
        }
        T* orow = out + (int64_t)i * pitch;
        if (j0 >= 1 && j0 + V - 1 <= cols) {
            VT v;
            T* e = (T*)&v;
#pragma unroll
            for (int x = 0; x < V; ++x) e[x] = r[x];
            *(VT*)(orow + j0) = v;
        } else if (inrow) {
#pragma unroll
            for (int x = 0; x < V; ++x)
                if (j0 + x >= 1 && j0 + x <= cols) orow[j0 + x] = r[x];
        }
    }
}

// Copies the interior of src into dst (used when an odd number of one-step
// launches leaves the result in the workspace).
template <typename T>
__global__ __launch_bounds__(256) void k_copy_interior(const T* __restrict__ src, T* __restrict__ dst,
                                                       int64_t pitch, int rows, int cols)
{
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i = blockIdx.y * 4 + threadIdx.y + 1;
    if (j <= cols && i <= rows) dst[(int64_t)i * pitch + j] = src[(int64_t)i * pitch + j];
}

// Copies the halo ring of src into dst (so a one-step workspace sees the grid's boundary).
template <typename T>
__global__ __launch_bounds__(256) void k_copy_halo(const T* __restrict__ src, T* __restrict__ dst,
                                                   int64_t pitch, int rows, int cols)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const int nrow = cols + 2, ncol = rows;
    if (idx < nrow) {
        dst[idx] = src[idx];
        dst[(int64_t)(rows + 1) * pitch + idx] = src[(int64_t)(rows + 1) * pitch + idx];
    } else if (idx < nrow + ncol) {
        const int64_t i = idx - nrow + 1;
        dst[i * pitch] = src[i * pitch];
        dst[i * pitch + cols + 1] = src[i * pitch + cols + 1];
    }
}

// Zeroes the sweep's barrier counters (kBarrierSlots slots, kFlagStride apart).
__global__ void k_reset_counter(uint32_t* bar)
{
    if (threadIdx.x < kBarrierSlots) __hip_atomic_store(bar + (size_t)threadIdx.x * kFlagStride, 0u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
}


// ============================================================================ host-side launchers

template <typename T>
static hipError_t launch_step9_t(bool fma, const void* in, void* out, int64_t pitch, int rows, int cols,
                                 const double* coeffs, hipStream_t st)
{
    Coef9<T> k;
    for (int q = 0; q < 9; ++q) k.k[q] = (T)coeffs[q];
    constexpr int V = 16 / (int)sizeof(T);
    if ((uintptr_t)in % 16 == 0 && (uintptr_t)out % 16 == 0 && pitch % V == 0) {
        dim3 grid((unsigned)((cols + 2 + 64 * V - 1) / (64 * V)), (unsigned)((rows + 4 * kStepRows - 1) / (4 * kStepRows)));
        if (fma) hipLaunchKernelGGL((k_step9_vec<T, true>), grid, dim3(256), 0, st, (const T*)in, (T*)out, pitch, rows, cols, k);
        else hipLaunchKernelGGL((k_step9_vec<T, false>), grid, dim3(256), 0, st, (const T*)in, (T*)out, pitch, rows, cols, k);
        return hipGetLastError();
    }
    dim3 block(64, 4);
    dim3 grid((cols + 63) / 64, (rows + 4 * kStepIlp - 1) / (4 * kStepIlp));
    if (fma) hipLaunchKernelGGL((k_step9<T, true>), grid, block, 0, st, (const T*)in, (T*)out, pitch, rows, cols, k);
    else hipLaunchKernelGGL((k_step9<T, false>), grid, block, 0, st, (const T*)in, (T*)out, pitch, rows, cols, k);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_step_t(bool fma, const void* in, void* out, int64_t pitch, int rows, int cols,
                                const double* coeffs, hipStream_t st)
{
    Coef<T> k{(T)coeffs[0], (T)coeffs[1], (T)coeffs[2], (T)coeffs[3], (T)coeffs[4]};
    constexpr int V = 16 / (int)sizeof(T);
    if ((uintptr_t)in % 16 == 0 && (uintptr_t)out % 16 == 0 && pitch % V == 0) {
        dim3 grid((unsigned)((cols + 2 + 64 * V - 1) / (64 * V)), (unsigned)((rows + 4 * kStepRows - 1) / (4 * kStepRows)));
        if (fma) hipLaunchKernelGGL((k_step_vec<T, true>), grid, dim3(256), 0, st, (const T*)in, (T*)out, pitch, rows, cols, k);
        else hipLaunchKernelGGL((k_step_vec<T, false>), grid, dim3(256), 0, st, (const T*)in, (T*)out, pitch, rows, cols, k);
        return hipGetLastError();
    }
    dim3 block(64, 4);
    dim3 grid((cols + 63) / 64, (rows + 4 * kStepIlp - 1) / (4 * kStepIlp));
    if (fma) hipLaunchKernelGGL((k_step<T, true>), grid, block, 0, st, (const T*)in, (T*)out, pitch, rows, cols, k);
    else hipLaunchKernelGGL((k_step<T, false>), grid, block, 0, st, (const T*)in, (T*)out, pitch, rows, cols, k);
    return hipGetLastError();
}

hipError_t launch_step(int dtype, bool fma, const void* in, void* out, int64_t pitch, int rows, int cols,
                       const double* coeffs, hipStream_t st, int pts)
{
    if (pts == 9)
        return dtype == 0 ? launch_step9_t<double>(fma, in, out, pitch, rows, cols, coeffs, st)
                          : launch_step9_t<float>(fma, in, out, pitch, rows, cols, coeffs, st);
    return dtype == 0 ? launch_step_t<double>(fma, in, out, pitch, rows, cols, coeffs, st)
                      : launch_step_t<float>(fma, in, out, pitch, rows, cols, coeffs, st);
}

hipError_t launch_copy_interior(int dtype, const void* src, void* dst, int64_t pitch, int rows, int cols,
                                hipStream_t st)
{
    dim3 block(64, 4);
    dim3 grid((cols + 63) / 64, (rows + 3) / 4);
    if (dtype == 0) hipLaunchKernelGGL((k_copy_interior<double>), grid, block, 0, st, (const double*)src, (double*)dst, pitch, rows, cols);
    else hipLaunchKernelGGL((k_copy_interior<float>), grid, block, 0, st, (const float*)src, (float*)dst, pitch, rows, cols);
    return hipGetLastError();
}

hipError_t launch_copy_halo(int dtype, const void* src, void* dst, int64_t pitch, int rows, int cols,
                            hipStream_t st)
{
    const int n = cols + 2 + rows;
    dim3 grid((n + 255) / 256);
    if (dtype == 0) hipLaunchKernelGGL((k_copy_halo<double>), grid, dim3(256), 0, st, (const double*)src, (double*)dst, pitch, rows, cols);
    else hipLaunchKernelGGL((k_copy_halo<float>), grid, dim3(256), 0, st, (const float*)src, (float*)dst, pitch, rows, cols);
    return hipGetLastError();
}

// Instantiated DTB kernels (one translation unit each, dtb_inst_*.hip): FP64
// with 2 columns per lane (R = 8, 16, 24) or 4 (R = 12), FP32 with 4, 8 waves
// per workgroup, R rows per lane.
#define DTB_DECLARE(NAME) const void* NAME(int kind, bool fma, bool colmask, bool rowcheck);
DTB_DECLARE(pick_f64c4_r12)
DTB_DECLARE(pick_f64w4_r24)
DTB_DECLARE(pick_f64_r8)
DTB_DECLARE(pick_f64_r16)
DTB_DECLARE(pick_f64_r24)
DTB_DECLARE(pick_f32_r8)
DTB_DECLARE(pick_f32_r16)
DTB_DECLARE(pick_f32_r24)
DTB_DECLARE(pick_f32_r28)
DTB_DECLARE(pick_box_f64_r8)
DTB_DECLARE(pick_box_f32_r16)
#undef DTB_DECLARE

// kind: 0 resident, 1 tile-serial sweep, 2 overlapped per-workgroup blocking.
// pts: 5 (j2d5pt) or 9 (the 3 x 3 box: FP64 4 x 8 and FP32 4 x 16 per lane,
// resident and sweep kernels only).
static const void* dtb_kernel_any(int kind, int dtype, int R, int want_waves, bool fma, bool colmask, bool rowcheck,
                                  int* C, int* waves, int pts)
{
    if (pts == 9) {
        if (want_waves != 0 && want_waves != 8) return nullptr;
        *waves = 8;
        *C = 4;
        if (kind == 2) return nullptr;
        if (dtype == 0 && R == 8) return pick_box_f64_r8(kind, fma, colmask, rowcheck);
        if (dtype == 1 && R == 16) return pick_box_f32_r16(kind, fma, colmask, rowcheck);
        return nullptr;
    }
    if (pts != 5) return nullptr;
    if (want_waves == 4) {
        // Half-height workgroups, two per compute unit (resident path only).
        *waves = 4;
        *C = 2;
        if (kind == 0 && dtype == 0 && R == 24) return pick_f64w4_r24(kind, fma, colmask, rowcheck);
        return nullptr;
    }
    if (want_waves != 0 && want_waves != 8) return nullptr;
    *waves = 8;
    if (dtype == 0) {
        *C = 2;
        switch (R) {
        case 8: return pick_f64_r8(kind, fma, colmask, rowcheck);
        case 16: return pick_f64_r16(kind, fma, colmask, rowcheck);
        case 24: return pick_f64_r24(kind, fma, colmask, rowcheck);
        case 12: *C = 4; return pick_f64c4_r12(kind, fma, colmask, rowcheck);
        default: return nullptr;
        }
    } else {
        *C = 4;
        switch (R) {
        case 8: return pick_f32_r8(kind, fma, colmask, rowcheck);
        case 16: return pick_f32_r16(kind, fma, colmask, rowcheck);
        case 24: return pick_f32_r24(kind, fma, colmask, rowcheck);
        case 28: return pick_f32_r28(kind, fma, colmask, rowcheck);
        default: return nullptr;
        }
    }
}

const void* dtb_kernel(int dtype, int R, bool fma, bool colmask, bool rowcheck, int* C, int* waves, int want_waves,
                       int pts)
{
    return dtb_kernel_any(0, dtype, R, want_waves, fma, colmask, rowcheck, C, waves, pts);
}

const void* dtb_sweep_kernel(int dtype, int R, bool fma, bool colmask, bool rowcheck, int* C, int* waves, int pts)
{
    return dtb_kernel_any(1, dtype, R, 8, fma, colmask, rowcheck, C, waves, pts);
}

const void* dtb_ovl_kernel(int dtype, int R, bool fma, bool colmask, bool rowcheck, int* C, int* waves)
{
    return dtb_kernel_any(2, dtype, R, 8, fma, colmask, rowcheck, C, waves, 5);
}

hipError_t launch_reset_counter(uint32_t* bar, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, bar);
    return hipGetLastError();
}

}  // namespace dtb
