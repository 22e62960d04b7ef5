// Specialised 3-mode MTTKRP kernel instantiations: FP32 factors, FP32
// accumulation (into the output or per-XCD copies).
#include "mttkrp_kernels.h"

namespace alto {

const void *pick_fast_f32(int lpn, int tile_merge) { return pick_fast<float, false>(lpn, tile_merge); }

}  // namespace alto
