// dtb_inst_box_f64_r8.hip -- the deep-temporal-blocking kernels for the 3 x 3 box stencil (j2d9pt), FP64,
// 4 columns x 8 rows per lane (a 64 x 256 register tile: the box's three-row working set leaves no room
// for the taller tiles of the 5-point stencil).
#include "dtb_tile.h"

namespace dtb {

const void* pick_box_f64_r8(int kind, bool fma, bool colmask, bool rowcheck)
{
    return pick_instance<double, 4, 8, kDtbWaves, false, 9>(kind, fma, colmask, rowcheck);
}

}  // namespace dtb
