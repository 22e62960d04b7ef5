// Specialised 3-mode MTTKRP kernel instantiations: BF16 factors.
#include "mttkrp_kernels.h"

namespace alto {

const void *pick_fast_bf16(int lpn, int tile_merge) { return pick_fast<uint16_t>(lpn, tile_merge); }

}  // namespace alto
