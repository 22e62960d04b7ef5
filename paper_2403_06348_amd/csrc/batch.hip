// Autotuning of the MTTKRP launch plan and batched MTTKRP.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "alto_internal.h"
#include "device_util.h"
#include "memory.h"
#include "mttkrp.h"

using namespace alto;

extern "C" {

alto_status alto_autotune(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors, float *out,
                          void *stream, alto_mttkrp_plan *chosen) {
    return fail(ALTO_ERR_ARG, "autotune not available yet");
}

alto_status alto_mttkrp_batched(int count, const alto_handle *hs, const int *modes, const int *ranks, const int *fdts,
                                const void *const *const *factors, float *const *outs, void *stream) {
    return fail(ALTO_ERR_ARG, "batched MTTKRP not available yet");
}

}  // extern "C"
