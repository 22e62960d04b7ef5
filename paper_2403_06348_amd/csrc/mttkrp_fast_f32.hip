// Specialised 3-mode MTTKRP kernel instantiations: FP32 factors.
#include "mttkrp_kernels.h"

namespace alto {

const void *pick_fast_f32(int lpn, int tile_merge) { return pick_fast<float>(lpn, tile_merge); }

}  // namespace alto
