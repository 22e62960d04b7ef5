// MTTKRP kernel instantiations: FP32 factors, 2-word ALTO index.
#include "mttkrp_kernels.h"

namespace alto {

const void *pick_lpn_f32_w2(int lpn, int nmodes, bool batch) { return pick_lpn<float, 2>(lpn, nmodes, batch); }

}  // namespace alto
