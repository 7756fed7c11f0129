// dtb_inst_f64_r8.hip -- the deep-temporal-blocking kernels for FP64, 2 columns x 8 rows per lane.
#include "dtb_tile.h"

namespace dtb {

const void* pick_f64_r8(int kind, bool fma, bool colmask, bool rowcheck)
{
    return pick_instance<double, 2, 8, kDtbWaves, true>(kind, fma, colmask, rowcheck);
}

}  // namespace dtb
