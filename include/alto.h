/*
 * alto.h -- C ABI of the MI355X (gfx950) ALTO sparse-tensor library.
 *
 * Implements, for one GPU, the hot path of "Accelerating Sparse Tensor
 * Decomposition Using Adaptive Linearized Representation" (Laukemann et al.,
 * arXiv 2403.06348):
 *   - ALTO format generation: linearization of every nonzero's coordinates
 *     into one bit-interleaved index (Sec. "ALTO Tensor Generation", Eq. 1,
 *     Fig. "alto_linear"(a)), ordering by that index, and partitioning of
 *     the ordered line into nnz-balanced segments with per-segment mode
 *     intervals (Sec. "Workload Partitioning and Scheduling");
 *   - MTTKRP on any mode over the single ALTO copy, with de-linearization by
 *     mask extraction (Fig. "alto_linear"(b)) and adaptive conflict
 *     resolution (Sec. "Adaptive Conflict Resolution");
 *   - one CP-ALS sweep (Algorithm "alg:cp-als").
 *
 * Conventions for every call
 *   - Pointers are DEVICE pointers unless marked "host".  Arrays of
 *     per-mode device pointers (coords, factors) are host arrays.
 *   - Coordinates and modes are 0-based.  Matrices are row-major.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on it; calls do not synchronize it
 *     unless stated.  A handle must not be used from two streams at once.
 *   - Every call returns an alto_status; on failure alto_last_error()
 *     (thread-local) describes it.  Argument errors are detected on the
 *     host before anything is enqueued.
 *   - Limits: 1 <= nmodes <= ALTO_MAX_MODES; 1 <= dims[n] <= 2^31; the
 *     index width sum_n ceil(log2 dims[n]) <= 128 bits; nnz < 2^40;
 *     rank 1..ALTO_MAX_RANK for MTTKRP and 1..64 for the CP-ALS calls (the
 *     R x R solve of a sweep runs in one workgroup's LDS).  A rank that is
 *     not a multiple of 4 runs on zero-padded copies of the factors (rows of
 *     the next multiple of 4) in handle workspace; the batched, serving and
 *     CP-APR calls take multiples of 4 only.
 */
#ifndef ALTO_MI355X_H
#define ALTO_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ALTO_MAX_MODES 8
#define ALTO_MAX_RANK 128

typedef struct alto_tensor *alto_handle;

typedef enum {
    ALTO_OK = 0,
    ALTO_ERR_ARG = 1,          /* invalid argument (detected on the host)            */
    ALTO_ERR_COORD_RANGE = 2,  /* a coordinate lies outside [0, dims[n])              */
    ALTO_ERR_INDEX_BITS = 3,   /* sum of index bits exceeds 128                       */
    ALTO_ERR_OOM = 4,          /* device allocation failed                            */
    ALTO_ERR_HIP = 5,          /* a HIP runtime call failed                           */
    ALTO_ERR_NOT_SPD = 6,      /* WARNING: V was not positive definite for at least   */
                               /* one mode; the pseudo-inverse was used, results valid */
    ALTO_ERR_STATE = 7,        /* handle not usable (NULL, freed, wrong object)       */
    ALTO_ERR_BUDGET = 8        /* serving: job can never fit the memory budget        */
} alto_status;

typedef enum { ALTO_F32 = 0, ALTO_BF16 = 1 } alto_dtype;

/* Conflict resolution of MTTKRP updates (Sec. "Adaptive Conflict Resolution").
 * ALTO_CR_TILE: updates of a tile of consecutive nonzeros are merged per output
 *   row in LDS (the GPU form of the per-partition temporary rows), then each
 *   merged row is added to the output once.
 * ALTO_CR_RUN: runs of consecutive nonzeros with the same output row are merged
 *   in registers and added to the output directly (the GPU form of the
 *   output-oriented traversal with atomics only where rows are shared).
 * ALTO_CR_DIRECT: for short modes, every output row of the mode (one rank tile
 *   of it) is held in LDS for the workgroup's whole line segment and added to
 *   the output once at its end (the paper's temporary rows indexed by the mode
 *   interval, which then spans the whole mode).
 * ALTO_CR_HOT: each workgroup picks the rows its line segment updates most
 *   often (from a strided sample of the segment) and merges their updates in
 *   LDS for the whole segment, adding each to the output once at its end;
 *   updates of all other rows merge in registers and go to the output
 *   directly.  The paper's temporary rows restricted to the segment's
 *   high-reuse rows (tensors of up to 5 modes).
 * ALTO_CR_AUTO: chosen per mode from the fiber reuse nnz / dims[mode]. */
typedef enum {
    ALTO_CR_AUTO = 0,
    ALTO_CR_TILE = 1,
    ALTO_CR_RUN = 2,
    ALTO_CR_DIRECT = 3,
    ALTO_CR_HOT = 4
} alto_conflict;

/* Where the merged output rows are summed.
 * ALTO_ACC_F64: in an FP64 buffer (handle workspace), rounded once to FP32.
 * ALTO_ACC_F32: directly in the FP32 output with FP32 atomics.
 * ALTO_ACC_XCD_F32 / ALTO_ACC_XCD_F64: in one private FP32 / FP64 copy of the
 *   output per XCD (the chiplet a workgroup runs on), summed in FP64 and
 *   rounded once to FP32 at the end; atomics of different XCDs never meet.
 * ALTO_ACC_DEFAULT (0): the library's accuracy policy.  FP32 atomics only
 *   where an output entry can take at most 256 additions (each can round
 *   away up to half a unit in the last place of the entry's running sum);
 *   else FP64: per-XCD copies for short modes with at least 512 nonzeros per
 *   row whose 8 copies take at most 1 GiB, otherwise one buffer (the
 *   autotuner times both).  Every entry then stays within 1e-5 of the sum of
 *   its terms' magnitudes. */
typedef enum {
    ALTO_ACC_DEFAULT = 0,
    ALTO_ACC_F64 = 1,
    ALTO_ACC_F32 = 2,
    ALTO_ACC_XCD_F32 = 3,
    ALTO_ACC_XCD_F64 = 4
} alto_accumulate;

/* Order in which the workgroups of a launch take the tiles (Sec. "Workload
 * Partitioning and Scheduling": nnz-balanced line segments per worker).
 * The tiles are split into one contiguous range per XCD either way.
 * ALTO_ORDER_CONTIGUOUS: each workgroup takes a contiguous stretch of its
 *   XCD's range (rows that recur in neighbouring tiles stay in its LDS table).
 * ALTO_ORDER_INTERLEAVED: the XCD's workgroups take its tiles round-robin, so
 *   the tiles in flight on one XCD are neighbours on the line and share L2
 *   lines of factor and output rows (TILE, RUN and DIRECT plans; HOT plans
 *   always use stretches).
 * ALTO_ORDER_DEFAULT (0): contiguous unless the autotuner recorded otherwise. */
typedef enum {
    ALTO_ORDER_DEFAULT = 0,
    ALTO_ORDER_CONTIGUOUS = 1,
    ALTO_ORDER_INTERLEAVED = 2
} alto_tile_order;

/* Tunable launch plan of one MTTKRP.  Zero fields take the library default
 * (or the autotuned value when one was recorded for the handle and mode). */
typedef struct {
    int conflict;        /* alto_conflict                                          */
    int tile_nnz;        /* nonzeros per workgroup tile (line segment length)      */
    int block_threads;   /* 256 or 512                                             */
    int table_slots;     /* LDS merge-table rows (power of two), TILE and HOT      */
    int accumulate;      /* alto_accumulate                                        */
    int rank_tile;       /* columns per pass (multiple of 4 dividing rank; 0: all) */
    int tile_order;      /* alto_tile_order: which tiles a workgroup takes          */
} alto_mttkrp_plan;

/* Host-side description of a handle (see alto_info). */
typedef struct {
    int nmodes;
    int index_bits;        /* B = sum_n ceil(log2 dims[n])                           */
    int index_words;       /* 1 (B <= 64) or 2 (64 < B <= 128) 64-bit words          */
    int nbits[ALTO_MAX_MODES];
    uint64_t dims[ALTO_MAX_MODES];
    uint64_t mask_lo[ALTO_MAX_MODES];  /* bits of the index holding mode n        */
    uint64_t mask_hi[ALTO_MAX_MODES];
    uint64_t nnz;
    uint64_t device_bytes; /* device memory owned by the handle right now          */
} alto_info_t;

/* ---------------------------------------------------------------- format */

/*
 * Plan only (host, no GPU needed): bit layout of the ALTO index for `dims`.
 * Mode n gets ceil(log2 dims[n]) bits; bit group l holds bit l of every mode
 * with more than l bits, shortest mode lowest (Sec. "ALTO Tensor
 * Generation", Eq. 1).  Fills every field of *out except nnz/device_bytes.
 * Errors: ALTO_ERR_ARG, ALTO_ERR_INDEX_BITS.
 */
alto_status alto_plan_dims(int nmodes, const uint64_t *dims /*host[nmodes]*/, alto_info_t *out /*host*/);

/*
 * Host reference of the extraction used on the device: decodes `count` ALTO
 * indices keys[2*i], keys[2*i+1] (lo, hi words; host) into coords[n*count+i]
 * (host, int64) with the same compiled code path as the GPU kernels.
 */
alto_status alto_plan_decode_host(const alto_info_t *plan, uint64_t count, const uint64_t *keys /*host*/,
                                  int64_t *coords /*host*/);

/*
 * Build an ALTO tensor (Sec. "ALTO Tensor Generation"): linearize every
 * nonzero, order the nonzeros by ALTO index (stable radix sort on the GPU)
 * and partition the line.  coords[n] is a device array of nnz int64
 * coordinates of mode n, vals a device array of nnz FP32 values.  The
 * library copies what it needs; the caller may free its inputs once the
 * stream has passed this call.  Duplicate coordinates stay separate
 * nonzeros.  nnz = 0 is valid.
 * Synchronizes `stream` once at the end to read the device coordinate-range
 * flag.  Errors: ALTO_ERR_ARG, ALTO_ERR_INDEX_BITS, ALTO_ERR_COORD_RANGE (no
 * handle is returned), ALTO_ERR_OOM, ALTO_ERR_HIP.
 */
alto_status alto_build(int nmodes, const uint64_t *dims /*host[nmodes]*/, uint64_t nnz,
                       const int64_t *const *coords /*host[nmodes] of device ptrs*/, const float *vals,
                       void *stream, alto_handle *out /*host*/);

/* Host description of a built tensor. */
alto_status alto_info(alto_handle h, alto_info_t *out /*host*/);

/*
 * Copy the ordered ALTO tensor out: keys_out gets nnz * index_words uint64
 * (word w of nonzero x at keys_out[x*index_words + w], low word first),
 * vals_out gets nnz FP32 values in the same order.  Either may be NULL.
 */
alto_status alto_export(alto_handle h, uint64_t *keys_out, float *vals_out, void *stream);

/*
 * De-linearize `count` ALTO indices (device, layout as in alto_export) with
 * the handle's masks (Fig. "alto_linear"(b)): coords_out[n*count + i]
 * (device int64).
 */
alto_status alto_decode(alto_handle h, uint64_t count, const uint64_t *keys, int64_t *coords_out, void *stream);

/*
 * Partition the ordered line into nseg nnz-balanced segments (Sec.
 * "Workload Partitioning and Scheduling"): starts_out[l] = floor(l*nnz/nseg)
 * for l = 0..nseg (device int64), and the closed mode intervals of every
 * segment, intervals_out[(l*nmodes + n)*2 + 0/1] = min/max mode-n
 * coordinate (device uint64); an empty segment gets (UINT64_MAX, 0).
 */
alto_status alto_partition(alto_handle h, int64_t nseg, int64_t *starts_out, uint64_t *intervals_out,
                           void *stream);

/*
 * Release the handle.  Its buffers return to the library's cache behind the
 * work already enqueued on the last stream the handle was used with (an
 * event recorded there; nothing waits).  Work the caller enqueued for the
 * handle on other streams must have completed.
 */
alto_status alto_free(alto_handle h);

/* ---------------------------------------------------------------- MTTKRP */

/*
 * MTTKRP of mode `mode` (Algorithm "alg:cp-als", MTTKRP line; sequential
 * MTTKRP-ALTO algorithm): out = X_(mode) (A^(0) KRP ... A^(N-1)) with the
 * mode's own factor left out, i.e. for every nonzero x,
 *   out[i_mode(x), r] += val(x) * prod_{m != mode} A^(m)[i_m(x), r].
 * factors[m] (device, row-major dims[m] x rank, FP32 or BF16 per fdt;
 * factors[mode] is not read and may be NULL).  out (device FP32,
 * dims[mode] x rank) is overwritten.  Accumulation is FP32 (partial rows) with
 * the final per-row sum in FP32 or FP64 per plan.  May allocate handle
 * workspace on first use of a (mode, rank).
 */
alto_status alto_mttkrp(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors,
                        float *out, void *stream);

/* Same, with an explicit launch plan (NULL = defaults). */
alto_status alto_mttkrp_ex(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors,
                           float *out, const alto_mttkrp_plan *plan, void *stream);

/*
 * Allocation-free MTTKRP, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): alto_mttkrp_ex with FP64 accumulation (ALTO_ACC_F64), whose
 * accumulation buffer is a static device array of the library instead of
 * handle workspace.  Nothing is allocated: no hipMalloc, hipFree or
 * allocating library routine.  Limits: rank a multiple of 4 and
 * dims[mode] * rank <= 8,388,608 (the array holds 2^23 doubles, 64 MiB, on
 * every GPU the library runs on, until the process ends); larger requests
 * fail with ALTO_ERR_ARG.  plan->accumulate must be 0 or ALTO_ACC_F64.  The
 * handle's device must be the current device.  All calls on one GPU share
 * the array: calls that overlap in time on one GPU (other streams, other
 * threads) race and give wrong results; calls on one stream are ordered.
 * The array is cleared by each call before use.
 */
alto_status alto_mttkrp_noalloc(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors,
                                float *out, const alto_mttkrp_plan *plan, void *stream);

/* Plan that alto_mttkrp would use for (mode, rank, fdt) (host). */
alto_status alto_mttkrp_get_plan(alto_handle h, int mode, int rank, alto_dtype fdt, alto_mttkrp_plan *out);

/*
 * Autotune (project-written): times candidate plans for (mode, rank, fdt) on
 * `stream` with the given factors (out is used as scratch and ends with a
 * valid result), records the fastest in the handle and in the process-wide
 * cache keyed by (nmodes, rank, index words, fdt, reuse class), and returns it.
 * Synchronizes the stream.
 */
alto_status alto_autotune(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors,
                          float *out, void *stream, alto_mttkrp_plan *chosen /*host, may be NULL*/);

/*
 * Many MTTKRPs in one persistent launch: item j computes MTTKRP of mode
 * modes[j] of handle hs[j] with rank ranks[j] and factor type fdts[j] from
 * factors[j][*] into outs[j].  Handles may differ in order, dims, index width
 * and nnz; all items' tiles form one work list that resident workgroups
 * drain.  Results are those of alto_mttkrp up to FP32 summation order.
 */
alto_status alto_mttkrp_batched(int count, const alto_handle *hs /*host*/, const int *modes /*host*/,
                                const int *ranks /*host*/, const int *fdts /*host*/,
                                const void *const *const *factors /*host[count] of host[nmodes]*/,
                                float *const *outs /*host[count]*/, void *stream);

/* ---------------------------------------------------------------- CP-APR */

/*
 * CP-APR model update of mode `mode` (Algorithm "alg:cp-apr-mu", the Phi
 * line; Algorithm "fig:subproblem_algo"):
 *   Phi(i, :) = sum over nonzeros x with i_mode(x) = i of
 *               val(x) / max(B(i, :) . krp_x, eps) * krp_x,
 * krp_x = Hadamard product of the other factors' rows A^(m)(i_m(x), :) --
 * the rows of the Khatri-Rao product Pi that the nonzeros need.
 * pi == NULL: krp is formed on the fly from `factors` (ALTO-OTF: factors[m]
 * device FP32 dims[m] x rank for m != mode).  Otherwise pi (device FP32,
 * nnz x rank, row x = krp of the x-th nonzero of the ordered line, from
 * alto_cpapr_pi) is read instead (ALTO-PRE; factors may be NULL; needs
 * nnz < 2^32).  B: device FP32 dims[mode] x rank; phi: device FP32
 * dims[mode] x rank, overwritten.  eps > 0.  rank: multiple of 4 in 4..128,
 * whole rank in one pass (the dot product needs every column); tensors of up
 * to 5 modes.  plan: as for alto_mttkrp_ex (NULL = the mode's MTTKRP plan,
 * adapted: no rank tiles, tables shrunk to fit).
 */
alto_status alto_cpapr_phi(alto_handle h, int mode, int rank, const float *const *factors, const float *B, float eps,
                           const float *pi, float *phi, const alto_mttkrp_plan *plan, void *stream);

/*
 * Pi for mode `mode` restricted to the nonzeros (Algorithm "alg:cp-apr-mu",
 * Pi line), for ALTO-PRE: pi (device FP32, nnz x rank, caller-owned;
 * nnz * rank * 4 bytes) row x = Hadamard product of the other factors' rows
 * at the x-th nonzero of the ordered line.
 */
alto_status alto_cpapr_pi(alto_handle h, int mode, int rank, const float *const *factors, float *pi, void *stream);

/*
 * The ALTO-PRE / ALTO-OTF choice for mode `mode` (Sec. "Adaptive Memory
 * Management"): *pre (host) = 1 when the mode's fiber reuse nnz / dims[mode]
 * is low (<= 4, the conflict-resolution rule's threshold) and the other
 * factor matrices (rank columns, FP32) exceed twice the GPU's L2 over all
 * XCDs (the GPU's fast memory), else 0.  Host only.
 */
alto_status alto_cpapr_prefer_pre(alto_handle h, int mode, int rank, int *pre /*host*/);

/* ---------------------------------------------------------------- CP-ALS */

/*
 * One CP-ALS sweep (Algorithm "alg:cp-als", one pass of the outer loop):
 * for n = 0..N-1: V = Hadamard product of the Grams A^(m)T A^(m), m != n
 * (FP64); M = MTTKRP(n); A^(n) = M V^-1 via an FP64 Cholesky factorisation of
 * V (symmetric-eigen pseudo-inverse when V is not positive definite; the call
 * stays asynchronous, so it does not return ALTO_ERR_NOT_SPD: the fallback
 * sets bit n of the flags alto_sweep_flags reads, and cpd_als returns the
 * warning); lambda = column 2-norms of A^(n)
 * (FP64); columns of A^(n) divided by lambda (a zero column stays zero).
 * factors[m] (device FP32, dims[m] x rank) are updated in place; lambda
 * (device FP64 [rank]) receives the last mode's norms.  fdt = ALTO_BF16 makes
 * the MTTKRPs read BF16 (round-to-nearest-even) shadow copies of the factors,
 * kept in handle workspace and refreshed after every update; Grams, solve and
 * lambda stay FP64 from the FP32 masters.
 * Everything stays on the GPU; the call is graph-capturable after a first
 * call has allocated the workspace.
 */
alto_status cpd_als_sweep(alto_handle h, int rank, float *const *factors, double *lambda, void *stream);
alto_status cpd_als_sweep_ex(alto_handle h, int rank, alto_dtype fdt, float *const *factors, double *lambda,
                             void *stream);

/*
 * One CP-ALS sweep of each of `count` tensors at once: for every mode step n,
 * the MTTKRPs of the tensors below 2^20 nonzeros that have a mode n run in
 * one persistent launch per kernel variant (as alto_mttkrp_batched), and
 * each larger tensor's in a launch of its own with its mode's plan (FP32
 * atomics or one FP64 buffer, never per-XCD copies); the FP64 Grams, R x R
 * solves and normalisations of all tensors run as one launch per step.  Per
 * item as cpd_als_sweep_ex:
 * hs[j], ranks[j], fdts[j], factors[j] (host array of device pointers),
 * lambdas[j] (device [ranks[j]]).  Tensors may differ in order, dims and
 * rank.  Results equal separate sweeps up to FP32 summation order.
 */
alto_status cpd_als_sweep_batched(int count, const alto_handle *hs /*host*/, const int *ranks /*host*/,
                                  const int *fdts /*host*/, float *const *const *factors /*host[count]*/,
                                  double *const *lambdas /*host[count] of device ptrs*/, void *stream);

/*
 * A batched sweep prepared once and run many times (Algorithm "alg:cp-als",
 * the same sweep as cpd_als_sweep_batched; ranks multiples of 4, 4..64).
 * alto_sweep_batch_create checks the items, allocates every workspace the
 * sweep needs, resolves the MTTKRP plans (the first sight of a batch class
 * times a few plans on `stream`, as cpd_als_sweep_batched does), uploads the
 * per-job tables to device memory the batch owns, and synchronizes `stream`
 * once.  alto_sweep_batch_run then enqueues one sweep of every item with
 * kernel launches only -- no allocation, copy, memset or host
 * synchronisation -- so it can be captured in a HIP graph and replayed; each
 * run or replay updates the items' factors and lambdas in place, from
 * whatever they hold when it starts.  The batch keeps the factor and lambda
 * pointers, the handles and their workspaces: they must stay alive and in
 * place while the batch (or a graph captured from it) is used.  A run
 * returns ALTO_ERR_STATE, and a captured graph must not be replayed, once a
 * handle's workspace was reallocated by a larger call on that handle.
 * Items must be on the current device.  Runs on different streams must not
 * overlap (they share the handles' workspaces).
 * alto_sweep_batch_destroy releases the tables (after the last run's
 * stream has passed them); NULL is accepted.
 */
typedef struct alto_sweep_batch *alto_sweep_batch_t;
alto_status alto_sweep_batch_create(int count, const alto_handle *hs /*host*/, const int *ranks /*host*/,
                                    const int *fdts /*host*/, float *const *const *factors /*host[count]*/,
                                    double *const *lambdas /*host[count] of device ptrs*/, void *stream,
                                    alto_sweep_batch_t *out /*host*/);
alto_status alto_sweep_batch_run(alto_sweep_batch_t batch, void *stream);
alto_status alto_sweep_batch_destroy(alto_sweep_batch_t batch);

/*
 * ||X||_F^2 of the tensor (host double; synchronizes the stream).  Duplicate
 * coordinates count as one entry holding their sum: they are neighbours on
 * the ordered line, and the norm is the sum over runs of equal ALTO index of
 * the squared run sum (FP64, fixed order, computed once per handle).
 */
alto_status alto_tensor_norm2(alto_handle h, double *norm2 /*host*/, void *stream);

/*
 * Fit of a CP model, the quantity Algorithm "alg:cp-als" watches:
 * fit = 1 - ||X - Xhat||_F / ||X||_F with Xhat = sum_r lambda[r] a_r^(0) o ...
 * o a_r^(N-1), a_r^(m) column r of factors[m] (device FP32 dims[m] x rank;
 * BF16 shadows are read for the MTTKRP when fdt = ALTO_BF16), lambda device
 * FP64 [rank].  Evaluated as ||X||^2 + lambda^T (Hadamard of the Grams)
 * lambda - 2 sum_r lambda_r <M(:, r), A^(N-1)(:, r)>, M the MTTKRP of the last
 * mode.  *fit (host) receives the value; synchronizes the stream.
 */
alto_status alto_cp_fit(alto_handle h, int rank, alto_dtype fdt, float *const *factors, const double *lambda,
                        double *fit /*host*/, void *stream);

/*
 * CP-ALS (Algorithm "alg:cp-als"): CP-ALS sweeps on `factors` (in place) until
 * the fit changes by less than `tol` from one sweep to the next (the fit has
 * ceased to improve) or `max_sweeps` sweeps have run.  The fit after each
 * sweep comes from the sweep's own Grams, last-mode MTTKRP and lambda (no
 * extra MTTKRP).  fits (host [max_sweeps], may be NULL) receives the fit after
 * each sweep, *sweeps_done (host, may be NULL) the number of sweeps; lambda
 * (device FP64 [rank]) the last mode's weights.  Blocking: synchronizes the
 * stream once per sweep to read the fit.  Returns ALTO_ERR_NOT_SPD (results
 * valid) when any mode update used the pseudo-inverse fallback.
 */
alto_status cpd_als(alto_handle h, int rank, alto_dtype fdt, float *const *factors, double *lambda, int max_sweeps,
                    double tol, double *fits /*host*/, int *sweeps_done /*host*/, void *stream);

/*
 * Status flags of the last sweep on `stream` (host, synchronizes the stream):
 * bit n set when mode n used the pseudo-inverse fallback.
 */
alto_status alto_sweep_flags(alto_handle h, void *stream, uint32_t *flags /*host*/);

/*
 * CP-APR by multiplicative updates (Algorithm "alg:cp-apr-mu"), around the
 * Phi and Pi kernels above.  For each outer iteration k <= k_max and mode n:
 * S = kappa where k > 1, A^(n) < kappa_tol and the mode's last Phi exceeds 1
 * (else 0); B = (A^(n) + S) Lambda; then up to l_max inner iterations of
 * Phi = (X_(n) ./ max(B Pi, eps)) Pi^T, stopping when the KKT violation
 * max over entries of |min(B, 1 - Phi)| is below tau, else B = B * Phi;
 * finally lambda = the column sums of B and A^(n) = B Lambda^-1 (a zero
 * column stays zero).  The outer loop ends early when no mode needed an
 * update (*converged = 1).  Pi rows are precomputed per mode and outer
 * iteration (nnz x rank FP32 of handle workspace) where alto_cpapr_prefer_pre
 * says so, and also for tensors of 4 or more modes when l_max >= 5 and Pi
 * takes at most 32 GiB: one streamed Pi row per nonzero then replaces N-1
 * gathered factor rows in every inner iteration (measured on the 4-mode
 * 2e8-nonzero workload at rank 32: Phi 11.7-26.6 ms from Pi against
 * 17.0-26.5 ms on the fly, Pi 12.6 ms per mode); else Pi rows are formed on
 * the fly.  params->pi_form overrides the rule.
 * factors (host array of device FP32 dims[m] x rank, non-negative) and
 * lambda (device FP64 [rank]; the caller's initial weights, e.g. ones) are
 * updated in place.  rank a multiple of 4 in 4..128; up to 5 modes.
 * outer_done, inner_counts (host [k_max x nmodes]: Phi evaluations per outer
 * iteration and mode) and converged may be NULL.  Blocking: synchronizes the
 * stream once per inner iteration to read the KKT value.  B and Phi are FP32,
 * lambda and the reductions FP64.  Errors: ALTO_ERR_ARG for bad arguments.
 */
typedef struct {
    int k_max;         /* outer iterations at most                           */
    int l_max;         /* inner iterations per mode at most (10 in the paper) */
    double tau;        /* KKT tolerance                                      */
    double kappa;      /* inadmissible-zero adjustment                       */
    double kappa_tol;  /* factor entries below this may be inadmissible zeros */
    float eps;         /* divisor floor of Phi                               */
    int pi_form;       /* 0: the library's rule (below), 1: Pi precomputed   */
                       /* per mode and outer iteration (ALTO-PRE), 2: Pi rows */
                       /* formed on the fly (ALTO-OTF)                        */
} alto_cpapr_params;
alto_status alto_cpapr_mu(alto_handle h, int rank, float *const *factors /*host[N] of device ptrs*/,
                          double *lambda, const alto_cpapr_params *params /*host*/, int *outer_done /*host*/,
                          int *inner_counts /*host*/, int *converged /*host*/, void *stream);

/* ---------------------------------------------------------------- serving */

/*
 * Continuous-batching CP-ALS server (one per GPU; a native scheduler thread).
 * Jobs are admitted while their estimated HBM footprint (ALTO tensor, build
 * scratch, factors, BF16 shadows, sweep workspace) fits the free budget and
 * an active slot is free; admitted tensors stay resident.  The scheduler
 * runs rounds: one CP-ALS sweep of every active job with the MTTKRPs of all
 * jobs batched (cpd_als_sweep_batched) on its compute stream, while newly
 * admitted jobs are built on a second stream.  A job retires after `sweeps`
 * sweeps; its factors (in place) and lambda_out then hold the result.
 * Jobs whose footprint exceeds the whole budget are rejected
 * (ALTO_ERR_BUDGET in their completion record).  All pointers in a job are
 * device pointers owned by the caller and must stay valid until the job's
 * completion record has been polled.  The server reads and writes them on
 * its own streams with no ordering against the caller's streams: every
 * write that produces a job's inputs must have completed (e.g. the
 * producing stream synchronized) before alto_server_submit, and the
 * outputs may be read once the completion record has been polled.  Ranks
 * are multiples of 4 in 4..64 here (and in the batched calls).
 */
typedef struct alto_server *alto_server_t;

typedef struct {
    int nmodes;
    int rank;             /* multiple of 4, 4..64 */
    int sweeps;           /* >= 1 */
    int fdt;              /* alto_dtype of the MTTKRP factor reads */
    uint64_t dims[ALTO_MAX_MODES];
    uint64_t nnz;
    const int64_t *coords[ALTO_MAX_MODES];  /* device [nnz] each */
    const float *vals;                      /* device [nnz] */
    float *factors[ALTO_MAX_MODES];         /* device dims[m] x rank, in/out */
    double *lambda_out;                     /* device [rank] */
    uint64_t user_tag;
} alto_serve_job;

typedef struct {
    uint64_t submitted, admitted, completed, rejected, active, queued;
    uint64_t bytes_in_use, bytes_peak;  /* admitted footprint (estimate) */
    uint64_t sweeps_done, nnz_modes_done, rounds;
} alto_serve_stats;

typedef struct {
    uint64_t user_tag;
    int status;          /* ALTO_OK or the error of its build/sweep */
    int sweeps;          /* sweeps completed */
    double submit_s, admit_s, done_s;  /* seconds on the server's clock */
    double sweep_ms_sum, sweep_ms_max; /* durations of the rounds it ran in */
} alto_serve_done;

/* budget_bytes: admitted-footprint cap; max_active: concurrent jobs. */
alto_status alto_server_create(uint64_t budget_bytes, int max_active, alto_server_t *out /*host*/);
/* Queue a job (copied; thread-safe).  Returns at once. */
alto_status alto_server_submit(alto_server_t s, const alto_serve_job *job /*host*/);
/* Move up to `max` completion records into out[]; *n receives the count. */
alto_status alto_server_poll(alto_server_t s, alto_serve_done *out /*host*/, int max, int *n /*host*/);
alto_status alto_server_stats(alto_server_t s, alto_serve_stats *out /*host*/);
/* Block until every submitted job has completed or been rejected. */
alto_status alto_server_drain(alto_server_t s);
/* Per-sweep (job, round) latencies in ms, oldest first; *n = count copied. */
alto_status alto_server_sweep_latencies(alto_server_t s, double *out /*host*/, uint64_t max, uint64_t *n);
/* Stop the scheduler after draining and release everything. */
alto_status alto_server_destroy(alto_server_t s);
/* Estimated HBM footprint of a job (host, no GPU needed). */
alto_status alto_serve_footprint(const alto_serve_job *job /*host*/, uint64_t *bytes /*host*/);

/* ---------------------------------------------------------------- timing */

/*
 * Kernel timing for measurement tools.  While enabled (on != 0), every launch
 * of the main MTTKRP kernel (alto_mttkrp*, the sweeps and batched calls) is
 * bracketed by a pair of HIP events recorded on its launch stream.
 * alto_timing_read waits for the recorded events, returns the number of
 * launches and the sum of their durations in milliseconds, and clears the
 * record.  Enabling or disabling also clears it.
 */
alto_status alto_timing_enable(int on);
alto_status alto_timing_read(uint64_t *launches /*host*/, double *total_ms /*host*/);

/* Return every cached device block to the device (hipFree).  Synchronizes
 * the device first. */
alto_status alto_release_cached_memory(void);

/* ---------------------------------------------------------------- misc */

/* Thread-local description of the last failure (never NULL). */
const char *alto_last_error(void);

/* Library version string, e.g. "alto-mi355x 1.0 gfx950". */
const char *alto_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ALTO_MI355X_H */
