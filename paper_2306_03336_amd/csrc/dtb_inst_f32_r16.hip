// dtb_inst_f32_r16.hip -- the deep-temporal-blocking kernels for FP32, 4 columns x 16 rows per lane.
#include "dtb_tile.h"

namespace dtb {

const void* pick_f32_r16(int kind, bool fma, bool colmask, bool rowcheck)
{
    return pick_instance<float, 4, 16>(kind, fma, colmask, rowcheck);
}

}  // namespace dtb
