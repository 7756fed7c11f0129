// dtb_inst_f64c4_r12.hip -- the deep-temporal-blocking kernels for FP64, 4 columns x 12 rows per lane
// (a 96 x 256 register tile: one cross-lane move per cell instead of two, at the same register budget
// as 2 columns x 24 rows).
#include "dtb_tile.h"

namespace dtb {

const void* pick_f64c4_r12(int kind, bool fma, bool colmask, bool rowcheck)
{
    return pick_instance<double, 4, 12, kDtbWaves, true>(kind, fma, colmask, rowcheck);
}

}  // namespace dtb
