// dtb_launch.h -- host-side entry points into the kernels of dtb_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dtb {

hipError_t launch_step(int dtype, bool fma, const void* in, void* out, int64_t pitch, int rows, int cols,
                       const double* coeffs, hipStream_t st);
hipError_t launch_copy_interior(int dtype, const void* src, void* dst, int64_t pitch, int rows, int cols,
                                hipStream_t st);
hipError_t launch_copy_halo(int dtype, const void* src, void* dst, int64_t pitch, int rows, int cols,
                            hipStream_t st);

// The DTB kernel for (dtype, rows per lane R, variant), or nullptr when that R
// is not instantiated.  *C receives the columns per lane and *waves the waves
// per workgroup of the instance.
const void* dtb_kernel(int dtype, int R, bool fma, bool colmask, bool rowcheck, int* C, int* waves);

}  // namespace dtb
