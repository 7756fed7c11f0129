// dtb_inst_3d.hip -- the j3d7pt kernels: the streaming kernels (FP64 2 x 4, FP32 4 x 4 and 3 x 4 cells per lane
// and plane, 8 waves, K = 1, 2, 3 steps per launch, fused and exact arithmetic), the one-step baseline and the
// copies around them, with their host-side launchers.
#include "dtb_stream3d.h"

namespace dtb {

template <typename T, int C, int R, int K>
static const void* stream_pick(bool fma)
{
    return fma ? (const void*)&k_stream3d<T, C, R, K, kStreamWaves, true>
               : (const void*)&k_stream3d<T, C, R, K, kStreamWaves, false>;
}

// The streaming kernel for (dtype, steps per launch K, columns per lane: 0 = the default instance), or nullptr;
// *C, *R: the instance's cells per lane.  FP64 2 x 4; FP32 4 x 4 (the default) and 3 x 4 (its 192-column tiles
// cover some widths with fewer ring columns: 512 columns in three spans of 192 instead of three of 256).
const void* dtb_stream3d_kernel(int dtype, int K, bool fma, int cols_per_lane, int* C, int* R)
{
    *R = 4;
    if (dtype == 0) {
        *C = 2;
        if (cols_per_lane != 0 && cols_per_lane != 2) return nullptr;
        switch (K) {
        case 1: return stream_pick<double, 2, 4, 1>(fma);
        case 2: return stream_pick<double, 2, 4, 2>(fma);
        case 3: return stream_pick<double, 2, 4, 3>(fma);
        default: return nullptr;
        }
    }
    if (cols_per_lane == 3) {
        *C = 3;
        switch (K) {
        case 1: return stream_pick<float, 3, 4, 1>(fma);
        case 2: return stream_pick<float, 3, 4, 2>(fma);
        case 3: return stream_pick<float, 3, 4, 3>(fma);
        default: return nullptr;
        }
    }
    *C = 4;
    if (cols_per_lane != 0 && cols_per_lane != 4) return nullptr;
    switch (K) {
    case 1: return stream_pick<float, 4, 4, 1>(fma);
    case 2: return stream_pick<float, 4, 4, 2>(fma);
    case 3: return stream_pick<float, 4, 4, 3>(fma);
    default: return nullptr;
    }
}

// ---- one-step baseline and copies

// One step per launch, HBM to HBM: thread (tx, ty) owns column j and row i and marches kStep3Planes planes
// in z, keeping the cells below, at and above the current plane in registers; the four in-plane neighbours
// come from memory (cache hits).  Same products in the same order as the streaming kernel.
constexpr int kStep3Planes = 16;

template <typename T, bool FMA>
__global__ __launch_bounds__(256) void k_step3d(const T* __restrict__ in, T* __restrict__ out, int64_t pitch,
                                                int64_t plane_pitch, int depth, int rows, int cols, Coef7<T> k)
{
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i = blockIdx.y * 4 + threadIdx.y + 1;
    const int z0 = blockIdx.z * kStep3Planes + 1;
    if (j > cols || i > rows) return;
    const int64_t off = (int64_t)i * pitch + j;
    T bel = in[(int64_t)(z0 - 1) * plane_pitch + off];
    T mid = in[(int64_t)z0 * plane_pitch + off];
    const int z1 = z0 + kStep3Planes - 1 < depth ? z0 + kStep3Planes - 1 : depth;
    for (int z = z0; z <= z1; ++z) {
        const T* p = in + (int64_t)z * plane_pitch + off;
        const T abv = p[plane_pitch];
        out[(int64_t)z * plane_pitch + off] = j3d7pt<FMA>(p[-1], p[1], p[-pitch], mid, p[pitch], bel, abv, k);
        bel = mid;
        mid = abv;
    }
}

// Copies the halo shell of src into dst: planes 0 and depth+1 whole, and rows 0 / rows+1 and columns 0 /
// cols+1 of every other plane (one thread per cell of the stored box; interior cells do nothing).
template <typename T>
__global__ __launch_bounds__(256) void k_copy_shell3d(const T* __restrict__ src, T* __restrict__ dst, int64_t pitch,
                                                      int64_t plane_pitch, int depth, int rows, int cols)
{
    const int64_t nx = cols + 2, ny = rows + 2, n = nx * ny * (depth + 2);
    for (int64_t t = blockIdx.x * (int64_t)256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
        const int64_t z = t / (nx * ny), rem = t % (nx * ny);
        const int64_t i = rem / nx, j = rem % nx;
        if (z == 0 || z == depth + 1 || i == 0 || i == rows + 1 || j == 0 || j == cols + 1) {
            const int64_t o = z * plane_pitch + i * pitch + j;
            dst[o] = src[o];
        }
    }
}

// Copies the interior of src into dst.
template <typename T>
__global__ __launch_bounds__(256) void k_copy_interior3d(const T* __restrict__ src, T* __restrict__ dst,
                                                         int64_t pitch, int64_t plane_pitch, int depth, int rows,
                                                         int cols)
{
    const int64_t n = (int64_t)cols * rows * depth;
    for (int64_t t = blockIdx.x * (int64_t)256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
        const int64_t z = t / ((int64_t)cols * rows) + 1, rem = t % ((int64_t)cols * rows);
        const int64_t o = z * plane_pitch + (rem / cols + 1) * pitch + rem % cols + 1;
        dst[o] = src[o];
    }
}

hipError_t launch_step3d(int dtype, bool fma, const void* in, void* out, int64_t pitch, int64_t plane_pitch,
                         int depth, int rows, int cols, const double* c, hipStream_t st)
{
    dim3 block(64, 4);
    dim3 grid((cols + 63) / 64, (rows + 3) / 4, (depth + kStep3Planes - 1) / kStep3Planes);
    if (dtype == 0) {
        Coef7<double> k{c[0], c[1], c[2], c[3], c[4], c[5], c[6]};
        if (fma) hipLaunchKernelGGL((k_step3d<double, true>), grid, block, 0, st, (const double*)in, (double*)out, pitch, plane_pitch, depth, rows, cols, k);
        else hipLaunchKernelGGL((k_step3d<double, false>), grid, block, 0, st, (const double*)in, (double*)out, pitch, plane_pitch, depth, rows, cols, k);
    } else {
        Coef7<float> k{(float)c[0], (float)c[1], (float)c[2], (float)c[3], (float)c[4], (float)c[5], (float)c[6]};
        if (fma) hipLaunchKernelGGL((k_step3d<float, true>), grid, block, 0, st, (const float*)in, (float*)out, pitch, plane_pitch, depth, rows, cols, k);
        else hipLaunchKernelGGL((k_step3d<float, false>), grid, block, 0, st, (const float*)in, (float*)out, pitch, plane_pitch, depth, rows, cols, k);
    }
    return hipGetLastError();
}

static unsigned copy_blocks(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

hipError_t launch_copy_shell3d(int dtype, const void* src, void* dst, int64_t pitch, int64_t plane_pitch, int depth,
                               int rows, int cols, hipStream_t st)
{
    const unsigned g = copy_blocks((int64_t)(cols + 2) * (rows + 2) * (depth + 2));
    if (dtype == 0) hipLaunchKernelGGL((k_copy_shell3d<double>), dim3(g), dim3(256), 0, st, (const double*)src, (double*)dst, pitch, plane_pitch, depth, rows, cols);
    else hipLaunchKernelGGL((k_copy_shell3d<float>), dim3(g), dim3(256), 0, st, (const float*)src, (float*)dst, pitch, plane_pitch, depth, rows, cols);
    return hipGetLastError();
}

hipError_t launch_copy_interior3d(int dtype, const void* src, void* dst, int64_t pitch, int64_t plane_pitch, int depth,
                                  int rows, int cols, hipStream_t st)
{
    const unsigned g = copy_blocks((int64_t)cols * rows * depth);
    if (dtype == 0) hipLaunchKernelGGL((k_copy_interior3d<double>), dim3(g), dim3(256), 0, st, (const double*)src, (double*)dst, pitch, plane_pitch, depth, rows, cols);
    else hipLaunchKernelGGL((k_copy_interior3d<float>), dim3(g), dim3(256), 0, st, (const float*)src, (float*)dst, pitch, plane_pitch, depth, rows, cols);
    return hipGetLastError();
}

}  // namespace dtb
