// Specialised 3-mode MTTKRP kernel instantiations: FP32 factors, FP64
// accumulation (one buffer or per-XCD copies).
#include "mttkrp_kernels.h"

namespace alto {

const void *pick_fast64_f32(int lpn, int tile_merge) { return pick_fast<float, true>(lpn, tile_merge); }

}  // namespace alto
