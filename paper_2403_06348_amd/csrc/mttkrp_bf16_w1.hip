// MTTKRP kernel instantiations: BF16 factors, 1-word ALTO index.
#include "mttkrp_kernels.h"

namespace alto {

const void *pick_lpn_bf16_w1(int lpn, int nmodes, bool batch) { return pick_lpn<uint16_t, 1>(lpn, nmodes, batch); }

}  // namespace alto
