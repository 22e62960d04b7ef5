// MTTKRP kernel instantiations: BF16 factors, 2-word ALTO index.
#include "mttkrp_kernels.h"

namespace alto {

const void *pick_lpn_bf16_w2(int lpn, int nmodes, bool batch) { return pick_lpn<uint16_t, 2>(lpn, nmodes, batch); }

}  // namespace alto
