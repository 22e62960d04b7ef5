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

// Project-written autotuner: times a small grid of launch plans around the
// default (tile length x LDS table rows, LDS-merged conflict resolution, plus
// direct atomics when fiber reuse is low) with HIP events on the caller's
// stream and keeps the fastest.  The result is recorded for the handle and
// in a process-wide cache keyed by the tensor's class, so later tensors of
// the same class skip the search.
alto_status alto_autotune(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors, float *out,
                          void *stream, alto_mttkrp_plan *chosen) {
    alto_status st = check_mttkrp_args(h, mode, rank, fdt, factors, out);
    if (st != ALTO_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const alto_mttkrp_plan base = default_plan(h, mode, rank, fdt);
    std::vector<alto_mttkrp_plan> cands;
    const uint64_t nnz = h->info.nnz;
    for (int tile : {2048, 4096, 8192, 16384, 32768}) {
        if (nnz > 0 && (uint64_t)tile * 64 > nnz && tile != base.tile_nnz) continue;  // keep >= 64 tiles
        for (int f : {1, 2, 4}) {
            alto_mttkrp_plan p = base;
            p.conflict = ALTO_CR_TILE;
            p.tile_nnz = tile;
            p.table_slots = std::max(64, base.table_slots * f / 2);
            if ((size_t)p.table_slots * (rank + 2) * 4 > 96 * 1024) continue;
            cands.push_back(p);
        }
    }
    const double reuse = nnz / (double)h->info.dims[mode];
    if (reuse <= 8.0) {
        alto_mttkrp_plan p = base;
        p.conflict = ALTO_CR_RUN;
        cands.push_back(p);
    }
    hipEvent_t e0, e1;
    ALTO_HIP(hipEventCreate(&e0));
    ALTO_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    alto_mttkrp_plan bestp = base;
    for (const auto &p : cands) {
        st = run_mttkrp(h, mode, rank, fdt, factors, out, p, s);  // warm
        if (st != ALTO_OK) break;
        ALTO_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 2; r++) {
            st = run_mttkrp(h, mode, rank, fdt, factors, out, p, s);
            if (st != ALTO_OK) break;
        }
        ALTO_HIP(hipEventRecord(e1, s));
        ALTO_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        ALTO_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            bestp = p;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ALTO_OK) return st;
    record_tuned(h, mode, rank, fdt, bestp);
    st = run_mttkrp(h, mode, rank, fdt, factors, out, bestp, s);
    if (st != ALTO_OK) return st;
    if (chosen) *chosen = bestp;
    return ALTO_OK;
}

alto_status alto_mttkrp_batched(int count, const alto_handle *hs, const int *modes, const int *ranks, const int *fdts,
                                const void *const *const *factors, float *const *outs, void *stream) {
    return fail(ALTO_ERR_ARG, "batched MTTKRP not available yet");
}

}  // extern "C"
