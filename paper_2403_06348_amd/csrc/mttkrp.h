// MTTKRP kernel arguments and host helpers shared by the MTTKRP, CP-ALS and
// batched translation units.
#pragma once

#include <string.h>

#include <vector>

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
    int lut;               // 1: 3 modes, one index word, <= 21 bits per mode (nibble-table decode)
    int interleave;        // 1: an XCD's workgroups take its tiles round-robin (with xcd_map)
    // CP-APR Phi forms: B (dims[mode] x ld FP32), Pi (nnz x ld FP32, ALTO
    // order; ALTO-PRE only), the divisor floor eps
    const float *phi_B;
    const float *phi_pi;
    float phi_eps;
};

constexpr int kXcdCopies = 8;  // XCDs of an MI355X

alto_mttkrp_plan default_plan(const alto_tensor *h, int mode, int rank, int fdt);
void record_tuned(alto_tensor *h, int mode, int rank, int fdt, const alto_mttkrp_plan &p);
alto_status resolve_plan(const alto_tensor *h, int mode, int rank, int fdt, const alto_mttkrp_plan *in,
                         alto_mttkrp_plan *out);
// FP32-atomic plans whose entries could take too many additions sum in FP64
// instead (one buffer or per-XCD copies; see mttkrp.hip); accumulate modes
// other than ALTO_ACC_F32 are left alone.
void accuracy_policy(const alto_tensor *h, int mode, int rank, alto_mttkrp_plan *p);
bool alternate_f64(const alto_tensor *h, int mode, int rank, alto_mttkrp_plan *p);
constexpr uint64_t kBatchF32MaxTiles = 256;  // batched launches (FP32 atomics): tiles per job at most
// Batched sweeps: a tensor of at least this many nonzeros takes its own
// MTTKRP launches (its mode's plan) instead of sharing the batched ones.
// Measured on a 256-job serving stream (offered load 0.7 / 4 of capacity):
// with the 512-thread default plans, 2^23 -> 2^20 cut the sweep latency p50
// from 10.6 to 1.9 ms and raised the saturated throughput from 6.5 to 9.8
// GNNZ/s (2^19 and 2^21 measured within 5% of 2^20).
constexpr uint64_t kBatchAloneNnz = uint64_t(1) << 20;
alto_status check_mttkrp_args(const alto_tensor *h, int mode, int rank, int fdt, const void *const *factors,
                              const float *out);
// Grow a workspace buffer to `need` bytes; a replaced buffer is released
// behind the work already enqueued on s (no synchronization).
alto_status ensure_ws(void **p, size_t *have, size_t need, hipStream_t s);
// acc_buf: accumulation buffer for FP64 / per-XCD plans (NULL: handle workspace)
alto_status run_mttkrp(alto_tensor *h, int mode, int rank, int fdt, const void *const *factors, float *out,
                       const alto_mttkrp_plan &p, hipStream_t s, void *acc_buf = nullptr);
void fill_args(const alto_tensor *h, int mode, int rank, int fdt, const void *const *factors,
               const alto_mttkrp_plan &p, float *out32, double *out64, MttkrpArgs *a, int col0 = 0,
               int rank_tile = 0);
size_t lds_bytes(const MttkrpArgs &a, int threads);
size_t outbox_bytes(int rank, int threads);  // per-wave outboxes of a launch
int lpn_for(int rank);
int pow2_floor(int v);
alto_status launch_mttkrp(const alto_tensor *h, int fdt, const MttkrpArgs &a, int threads, hipStream_t s);
// Persistent launch of a stretch kernel (grid = CUs x occupancy, XCD-ordered
// stretches), timed when timing is enabled.
alto_status launch_stretch_kernel(const alto_tensor *h, const void *kern, const MttkrpArgs &a, int threads,
                                  hipStream_t s);
// LDS bytes beyond the tables a stretch kernel may use (static arrays).
size_t static_lds_allowance();
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
size_t device_lds(int dev);  // LDS bytes one workgroup may allocate
size_t device_cache_bytes(int dev);  // L2 bytes over all XCDs

// batched MTTKRP (batch.hip), arguments already validated
alto_status batched_run(int count, const alto_handle *hs, const int *modes, const int *ranks, const int *fdts,
                        const void *const *const *factors, float *const *outs, hipStream_t s);

// One persistent launch of a kernel-variant group of a batched MTTKRP,
// planned on the host: the per-job kernel arguments and the tile and output
// prefixes, copied to the device as one blob (jobs, prefix, oprefix).
struct GroupLaunch {
    std::vector<MttkrpArgs> jobs;
    std::vector<uint64_t> prefix, oprefix;
    const void *kern = nullptr;
    size_t lds = 0;
    unsigned grid = 1;
    int nj = 0, xcd_map = 0, threads = 256;
    size_t jobs_bytes() const { return sizeof(MttkrpArgs) * (size_t)nj; }
    size_t prefix_bytes() const { return 8 * (size_t)(nj + 1); }
    size_t blob_bytes() const { return jobs_bytes() + 2 * prefix_bytes(); }
    void write_blob(char *dst) const {
        memcpy(dst, jobs.data(), jobs_bytes());
        memcpy(dst + jobs_bytes(), prefix.data(), prefix_bytes());
        memcpy(dst + jobs_bytes() + prefix_bytes(), oprefix.data(), prefix_bytes());
    }
};
// The groups of a batched MTTKRP with their tuned plans (the first sight of
// a group class runs and times a few plans on stream s).
alto_status batched_plan(int count, const alto_handle *hs, const int *modes, const int *ranks, const int *fdts,
                         const void *const *const *factors, float *const *outs, hipStream_t s,
                         std::vector<GroupLaunch> *out);
// Zero the group's outputs and launch it; dblob holds write_blob's bytes.
// Kernel launches only (capturable in a HIP graph).
alto_status launch_planned_group(const GroupLaunch &gl, const void *dblob, hipStream_t s);

// CP-APR (phi.hip): Phi of a mode into `phi` (dims[mode] x rank FP32) from
// B and the other factors, or from precomputed Pi rows (ALTO order); Pi rows
// of a mode; whether the PRE form is the better one for a mode.
alto_status run_phi(alto_tensor *h, int mode, int rank, const void *const *factors, const float *B, float eps,
                    const float *pi, float *phi, const alto_mttkrp_plan *in, hipStream_t s);
alto_status run_pi(alto_tensor *h, int mode, int rank, const float *const *factors, float *pi, hipStream_t s);
bool prefer_pre(const alto_tensor *h, int mode, int rank);

// Ranks that are not a multiple of 4: the library works on copies whose rows
// are padded with zero columns to the next multiple of 4 (mttkrp.hip).
inline int padded_rank(int rank) { return (rank + 3) & ~3; }
// dst (I x ldd) = src (I x lds) in columns [0, lds), zero in [lds, ldd);
// esize 2 or 4 bytes.  Also used the other way (ldd < lds) to copy back.
void launch_copy_cols(const void *src, int lds, void *dst, int ldd, uint64_t I, int esize, hipStream_t s);
// Zero-padded copies of factors[m] (m != skip) in the handle's pad
// workspace; fptr[m] receives them.
alto_status pad_factors(alto_tensor *h, int rank, int fdt, const void *const *factors, int skip, void **fptr,
                        hipStream_t s);

// The autotuner at a rank that is a multiple of 4 (batch.hip).
alto_status autotune_run(alto_tensor *h, int mode, int rank, int fdt, const void *const *factors, float *out,
                         hipStream_t s, alto_mttkrp_plan *chosen);

// CP-ALS sweep phases (als.hip)
alto_status sweep_begin(alto_tensor *h, int rank, int fdt, float *const *factors, const double *lambda, hipStream_t s);
void sweep_factor_ptrs(const alto_tensor *h, int fdt, float *const *factors, const void **fptr);
alto_status sweep_pre(alto_tensor *h, int n, int rank, int rank_true, hipStream_t s);
// One sweep at a rank that is a multiple of 4, of which the first rank_true
// columns are the model (the others zero padding).
alto_status sweep_run(alto_tensor *h, int rank, int rank_true, int fdt, float *const *factors, double *lambda,
                      hipStream_t s);
alto_status sweep_post(alto_tensor *h, int n, int rank, int fdt, float *const *factors, double *lambda,
                       hipStream_t s);
// CP fit (fit.hip): ||X||^2 once per handle into h->ws_fit[0]; the fit of the
// model left in the sweep workspace (Grams, last mode's MTTKRP in ws_m).
alto_status ensure_xnorm2(alto_tensor *h, hipStream_t s);
alto_status launch_fit(alto_tensor *h, int rank, const float *A_last, const double *lam, double *fit, hipStream_t s);
// Partial R x R Grams the sweep workspace holds (after the Grams and the
// solve operator); the fit's column dot products reuse that area.
constexpr int kSweepPartials = 512;
bool timing_begin(hipStream_t s, hipEvent_t *e0, hipEvent_t *e1);
void timing_end(hipStream_t s, hipEvent_t e0, hipEvent_t e1);

}  // namespace alto
