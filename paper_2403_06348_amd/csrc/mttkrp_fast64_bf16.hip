// Specialised 3-mode MTTKRP kernel instantiations: BF16 factors, FP64
// accumulation (one buffer or per-XCD copies).
#include "mttkrp_kernels.h"

namespace alto {

const void *pick_fast64_bf16(int lpn, int tile_merge) { return pick_fast<uint16_t, true>(lpn, tile_merge); }

}  // namespace alto
