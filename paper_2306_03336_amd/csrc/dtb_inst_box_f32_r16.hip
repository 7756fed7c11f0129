// dtb_inst_box_f32_r16.hip -- the deep-temporal-blocking kernels for the 3 x 3 box stencil (j2d9pt), FP32,
// 4 columns x 16 rows per lane (a 128 x 256 register tile).
#include "dtb_tile.h"

namespace dtb {

const void* pick_box_f32_r16(int kind, bool fma, bool colmask, bool rowcheck)
{
    return pick_instance<float, 4, 16, kDtbWaves, false, 9>(kind, fma, colmask, rowcheck);
}

}  // namespace dtb
