// dtb_inst_f64w4_r24.hip -- the deep-temporal-blocking kernels for FP64, 2 columns x 24 rows per lane,
// 4 waves per workgroup: a 96 x 128 register tile, two workgroups per compute unit, so that one
// workgroup's exchange overlaps the other's steps.
#include "dtb_tile.h"

namespace dtb {

const void* pick_f64w4_r24(int kind, bool fma, bool colmask, bool rowcheck)
{
    return pick_instance<double, 2, 24, 4>(kind, fma, colmask, rowcheck);
}

}  // namespace dtb
