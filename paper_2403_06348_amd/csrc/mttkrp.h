// MTTKRP kernel arguments and host helpers shared by the MTTKRP, CP-ALS and
// batched translation units.
#pragma once

#include "alto_internal.h"

namespace alto {

constexpr int kMaxProbe = 16;       // LDS table probes before falling back to the output
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr uint32_t kHotHits = 4;    // runs merged in one tile that make a row stay in LDS
constexpr int kKeepTiles = 16;      // tiles a row may stay in LDS before it is flushed

struct MttkrpArgs {
    LinePlan lp;
    const void *fac_other[ALTO_MAX_MODES];  // factors of the other modes, ascending mode order
    uint32_t last_other[ALTO_MAX_MODES];    // dims - 1 of those modes (gather index clamp)
    uint32_t dim_out;                       // dims[mode]
    uint32_t fac_bytes[ALTO_MAX_MODES];     // byte size of those factors (buffer range)
    int buf32;                              // 1: gathers through 32-bit buffer offsets
    const uint64_t *keys;
    const float *vals;
    float *out32;
    double *out64;
    uint64_t nnz;
    uint64_t ntiles;
    uint64_t tq, tr;  // nnz / ntiles, nnz % ntiles
    int mode, rank, nmodes;
    int tile_merge;   // 0: direct atomics, 1: LDS table merge, 2: whole mode in LDS
    int tw;           // 32-bit words per LDS table element: 2 = FP64, 1 = FP32
    int use64;        // 1: accumulate into out64
    int slots_log2;
    int rec;          // staged record length (u32) per nonzero
    int xcd_map;      // 1: contiguous tile ranges per XCD
    int copies;       // private output copies, indexed by XCD id (1: shared output)
    uint32_t ld;      // row stride of factors and output (the full rank)
    uint32_t col0;    // first column of this rank tile
    uint64_t copy_stride;  // elements per copy
};

constexpr int kXcdCopies = 8;  // XCDs of an MI355X

alto_mttkrp_plan default_plan(const alto_tensor *h, int mode, int rank, int fdt);
void record_tuned(alto_tensor *h, int mode, int rank, int fdt, const alto_mttkrp_plan &p);
alto_status resolve_plan(const alto_tensor *h, int mode, int rank, int fdt, const alto_mttkrp_plan *in,
                         alto_mttkrp_plan *out);
alto_status check_mttkrp_args(const alto_tensor *h, int mode, int rank, int fdt, const void *const *factors,
                              const float *out);
alto_status ensure_ws(void **p, size_t *have, size_t need);
alto_status run_mttkrp(alto_tensor *h, int mode, int rank, int fdt, const void *const *factors, float *out,
                       const alto_mttkrp_plan &p, hipStream_t s);
void fill_args(const alto_tensor *h, int mode, int rank, int fdt, const void *const *factors,
               const alto_mttkrp_plan &p, float *out32, double *out64, MttkrpArgs *a, int col0 = 0,
               int rank_tile = 0);
size_t lds_bytes(const MttkrpArgs &a, int threads);
int lpn_for(int rank);
int pow2_floor(int v);
alto_status launch_mttkrp(const alto_tensor *h, int fdt, const MttkrpArgs &a, int threads, hipStream_t s);
const void *pick_kernel(int lpn, int fdt, int words, int nmodes, bool batch);
const void *pick_single(int lpn, int fdt, int words, const MttkrpArgs &a);
// Largest whole-mode LDS table (bytes) a workgroup of `threads` can hold
// beside its record staging on this tensor's device.
size_t direct_table_limit(const alto_tensor *h, int threads);
// LDS bytes of a hashed-table plan (table, record staging, static LDS), and
// whether it fits one workgroup on this tensor's device.
size_t tile_plan_lds(const alto_tensor *h, int rank_tile, int slots, int threads);
bool tile_plan_fits(const alto_tensor *h, int rank_tile, int slots, int threads);
// ALTO_ERR_ARG when `dyn` bytes of dynamic LDS plus the kernel's static LDS
// exceed what a workgroup may allocate on device `dev`.
alto_status check_launch_lds(const void *kern, size_t dyn, int dev);
const void *zero_outputs_kernel();
int device_cus(int dev);

// batched MTTKRP (batch.hip), arguments already validated
alto_status batched_run(int count, const alto_handle *hs, const int *modes, const int *ranks, const int *fdts,
                        const void *const *const *factors, float *const *outs, hipStream_t s);

// CP-ALS sweep phases (als.hip)
alto_status sweep_begin(alto_tensor *h, int rank, int fdt, float *const *factors, const double *lambda, hipStream_t s);
void sweep_factor_ptrs(const alto_tensor *h, int fdt, float *const *factors, const void **fptr);
alto_status sweep_pre(alto_tensor *h, int n, int rank, hipStream_t s);
alto_status sweep_post(alto_tensor *h, int n, int rank, int fdt, float *const *factors, double *lambda,
                       hipStream_t s);
bool timing_begin(hipStream_t s, hipEvent_t *e0, hipEvent_t *e1);
void timing_end(hipStream_t s, hipEvent_t e0, hipEvent_t e1);

}  // namespace alto
