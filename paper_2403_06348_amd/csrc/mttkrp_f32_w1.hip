// MTTKRP kernel instantiations: FP32 factors, 1-word ALTO index.
#include "mttkrp_kernels.h"

namespace alto {

const void *pick_lpn_f32_w1(int lpn, int nmodes, bool batch) { return pick_lpn<float, 1>(lpn, nmodes, batch); }

}  // namespace alto
