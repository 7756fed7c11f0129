// dtb_inst_batch.hip -- the batched persistent kernel and the register-tile
// instances it carries: FP64 2 x 16 (128 x 128 tiles) and 4 x 8 (64 x 256);
// FP32 4 x 16 (128 x 256) and 4 x 8 (64 x 256).  Two shapes per precision at the
// same register budget per lane, so carrying both costs no registers.
#include "dtb_tile.h"

namespace dtb {

const void* batched_kernel(TileInst* insts, int* n)
{
    const TileInst list[] = {{0, kBatchR64a, kBatchC64a}, {0, kBatchR64b, kBatchC64b},
                             {1, kBatchR32a, kBatchC32a}, {1, kBatchR32b, kBatchC32b}};
    *n = 0;
    for (const TileInst& t : list) insts[(*n)++] = t;
    return (const void*)&k_dtb_batched<true>;
}

}  // namespace dtb
