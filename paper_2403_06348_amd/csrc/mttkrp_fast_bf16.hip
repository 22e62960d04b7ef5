// Specialised 3-mode MTTKRP kernel instantiations: BF16 factors, FP32
// accumulation (into the output or per-XCD copies).
#include "mttkrp_kernels.h"

namespace alto {

const void *pick_fast_bf16(int lpn, int tile_merge) { return pick_fast<uint16_t, false>(lpn, tile_merge); }

}  // namespace alto
