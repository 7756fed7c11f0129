// dtb_inst_batch.hip -- the batched persistent kernel (FP64: 2 x 16 per lane, FP32: 4 x 16).
#include "dtb_tile.h"

namespace dtb {

const void* batched_kernel(int* rows_per_lane_f64, int* rows_per_lane_f32)
{
    *rows_per_lane_f64 = 16;
    *rows_per_lane_f32 = 16;
    return (const void*)&k_dtb_batched<16, 16, true>;
}

}  // namespace dtb
