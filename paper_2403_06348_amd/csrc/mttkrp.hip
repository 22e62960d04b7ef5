// MTTKRP host side: launch plans, workspace, launches and the MTTKRP entry
// points of the C ABI.  The device code is in mttkrp_kernels.h.
#include <string.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "memory.h"
#include "mttkrp_kernels.h"

namespace alto {

// Kernel pointers, one translation unit per factor type and index width.
const void *pick_lpn_f32_w1(int lpn, int nmodes, bool batch);
const void *pick_lpn_f32_w2(int lpn, int nmodes, bool batch);
const void *pick_lpn_bf16_w1(int lpn, int nmodes, bool batch);
const void *pick_lpn_bf16_w2(int lpn, int nmodes, bool batch);
const void *pick_fast_f32(int lpn, int tile_merge);
const void *pick_fast_bf16(int lpn, int tile_merge);
const void *pick_fast64_f32(int lpn, int tile_merge);
const void *pick_fast64_bf16(int lpn, int tile_merge);

const void *pick_kernel(int lpn, int fdt, int words, int nmodes, bool batch) {
    if (fdt == ALTO_BF16)
        return words == 2 ? pick_lpn_bf16_w2(lpn, nmodes, batch) : pick_lpn_bf16_w1(lpn, nmodes, batch);
    return words == 2 ? pick_lpn_f32_w2(lpn, nmodes, batch) : pick_lpn_f32_w1(lpn, nmodes, batch);
}

// The specialised kernel serves 3-mode tensors with a one-word index whose
// factor reads fit 32-bit offsets; everything else takes the general kernel.
const void *pick_single(int lpn, int fdt, int words, const MttkrpArgs &a) {
    if (words == 1 && a.nmodes == 3 && a.buf32) {
        if (a.use64) return fdt == ALTO_BF16 ? pick_fast64_bf16(lpn, a.tile_merge) : pick_fast64_f32(lpn, a.tile_merge);
        return fdt == ALTO_BF16 ? pick_fast_bf16(lpn, a.tile_merge) : pick_fast_f32(lpn, a.tile_merge);
    }
    return pick_kernel(lpn, fdt, words, a.nmodes, false);
}

const void *zero_outputs_kernel() { return (const void *)k_zero_outputs; }

namespace {

struct DevProps {
    int cus = 0;
    size_t lds = 0;    // LDS bytes one workgroup may allocate
    size_t cache = 0;  // L2 bytes over all XCDs
};

DevProps &props(int dev);
}  // namespace

int device_cus(int dev) { return props(dev).cus; }
size_t device_lds(int dev) { return props(dev).lds; }
size_t device_cache_bytes(int dev) { return props(dev).cache; }

// Static LDS of the MTTKRP kernels (extraction masks, the nibble decode
// table, counters) is below this; plans budget it beside their tables and
// record staging.
constexpr size_t kStaticLdsAllowance = 4096;
size_t static_lds_allowance() { return kStaticLdsAllowance; }

// LDS words staged per nonzero: [value, destination, other coordinates]
// rounded to 16 bytes.
int record_words(int nmodes, int words) {
    (void)words;
    return (nmodes + 1 + 3) / 4 * 4;
}

// The per-wave outboxes of rows bound for the output (see the kernels):
// two slots per lane group, each a row index and `rank` FP32 columns.
size_t outbox_bytes(int rank, int threads) {
    const int cap = 2 * (64 / lpn_for(rank));
    return (size_t)(threads / 64) * cap * (rank + 1) * 4;
}

size_t tile_plan_lds(const alto_tensor *h, int rank_tile, int slots, int threads) {
    const size_t rec = (size_t)record_words(h->info.nmodes, h->info.index_words);
    return (size_t)slots * (2 * (rank_tile + 1) + 2) * 4 + (size_t)threads * rec * 4 + outbox_bytes(rank_tile, threads) +
           kStaticLdsAllowance;
}

bool tile_plan_fits(const alto_tensor *h, int rank_tile, int slots, int threads) {
    return tile_plan_lds(h, rank_tile, slots, threads) <= props(h->device).lds;
}

alto_status check_launch_lds(const void *kern, size_t dyn, int dev) {
    hipFuncAttributes fa;
    size_t stat = 256;
    if (hipFuncGetAttributes(&fa, kern) == hipSuccess) stat = fa.sharedSizeBytes;
    else (void)hipGetLastError();
    if (dyn + stat > props(dev).lds)
        return fail(ALTO_ERR_ARG, "launch needs " + std::to_string(dyn + stat) + " bytes of LDS; the device has " +
                                      std::to_string(props(dev).lds));
    return ALTO_OK;
}

size_t direct_table_limit(const alto_tensor *h, int threads) {
    const size_t rec = (size_t)record_words(h->info.nmodes, h->info.index_words);
    const size_t stage = (size_t)threads * rec * 4 + kStaticLdsAllowance;  // + static LDS and alignment
    const size_t lds = props(h->device).lds;
    return lds > stage ? lds - stage : 0;
}

namespace {

DevProps &props(int dev) {
    static DevProps p[64];
    if (dev >= 0 && dev < 64 && p[dev].cus == 0) {
        hipDeviceProp_t dp;
        if (hipGetDeviceProperties(&dp, dev) == hipSuccess) {
            p[dev].cus = dp.multiProcessorCount;
            p[dev].lds = dp.sharedMemPerBlock;
            // the runtime reports one XCD's L2
            p[dev].cache = (size_t)dp.l2CacheSize * kXcdCopies;
        } else {
            p[dev].cus = 256;
            p[dev].lds = 64 * 1024;
            p[dev].cache = size_t(32) << 20;
        }
    }
    return p[dev < 0 || dev >= 64 ? 0 : dev];
}

}  // namespace

int pow2_floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

int lpn_for(int rank) {
    int l = 1;
    while (4 * l < rank) l <<= 1;
    return l;
}

alto_mttkrp_plan default_plan(const alto_tensor *h, int mode, int rank, int fdt) {
    alto_mttkrp_plan p;
    memset(&p, 0, sizeof(p));
    const double reuse = (double)h->info.nnz / (double)h->info.dims[mode];
    // initial rule of the paper: buffered (tile) merging pays off when the
    // average number of nonzeros per output fiber exceeds the 4 memory
    // operations a buffered update costs in the worst case
    p.conflict = reuse > 4.0 ? ALTO_CR_TILE : ALTO_CR_RUN;
    // The defaults follow the autotuner's choices on 34 modes of eight
    // 0.9e7-2e7-nonzero Zipf tensors of 3-5 modes (R 8-32), where the former
    // defaults (256 threads, tiles growing to nnz/8192, FP32-row whole-mode
    // tables) ran 1.2-2x slower on most modes and up to 20x on short skewed
    // ones: 512 threads in 31 of 34 modes, tiles longer at lower rank.
    p.block_threads = 512;
    // LDS table of about 64 KiB of FP64 partial rows
    int slots = 8192 / rank;
    int s2 = 1;
    while (s2 * 2 <= slots) s2 *= 2;
    p.table_slots = std::max(64, s2);
    // long tiles amortize the table flush (the longer the lower the rank);
    // keep about 2048 tiles to fill the GPU
    const int tmax = std::min(16384, std::max(2048, pow2_floor(std::max(1, 131072 / rank))));
    uint64_t tile = 512;
    while (tile < (uint64_t)tmax && tile * 2048 < h->info.nnz) tile *= 2;
    p.tile_nnz = (int)tile;
    p.accumulate = ALTO_ACC_F32;
    // a mode short enough to hold whole in LDS in FP64 rows, in at most two
    // passes (rank tiles of at least 8 columns), is accumulated there for
    // the workgroup's whole segment.  FP32 rows (added by compare-and-swap)
    // are left to the autotuner: on skewed modes the swaps of hot rows retry
    // (5.0 and 9.4 ms against 0.8 and 0.5 ms for the table merge on two
    // such modes), on uniform ones they can win.
    const size_t lim = direct_table_limit(h, p.block_threads);
    int rt_d = 0;
    for (int rt = rank; rt >= 8 && rt % 4 == 0 && rank % rt == 0 && 2 * rt >= rank; rt /= 2) {
        if ((size_t)h->info.dims[mode] * (rt + 1) * 8 <= lim) {
            rt_d = rt;
            break;
        }
    }
    if (rt_d && reuse > 4.0) {
        p.conflict = ALTO_CR_DIRECT;
        p.rank_tile = rt_d == rank ? 0 : rt_d;
    }
    (void)fdt;
    return p;
}

// 32-bit words per whole-mode LDS row element of a plan on this tensor: FP64
// rows when the rank tile fits so, else FP32 rows (see fill_args).
int direct_row_words(const alto_tensor *h, int mode, int rank, const alto_mttkrp_plan &p) {
    const int rt = p.rank_tile > 0 ? p.rank_tile : rank;
    return (size_t)h->info.dims[mode] * (rt + 1) * 8 <= direct_table_limit(h, p.block_threads) ? 2 : 1;
}

// Tuned plans per tensor class, with the whole-mode row width the plan had
// where it was tuned.
struct CachedPlan {
    alto_mttkrp_plan p;
    int row_words;
};
static std::mutex g_tune_mu;
static std::map<std::array<int, 6>, CachedPlan> g_tune_cache;

std::array<int, 6> tune_key(const alto_tensor *h, int mode, int rank, int fdt) {
    const double reuse = (double)h->info.nnz / (double)h->info.dims[mode];
    const int lr = reuse > 0 ? (int)std::floor(std::log2(reuse)) : -64;
    const int ln = h->info.nnz > 0 ? (int)std::floor(std::log2((double)h->info.nnz)) : -1;
    return {h->info.nmodes, rank, h->info.index_words, fdt, lr, ln};
}

void record_tuned(alto_tensor *h, int mode, int rank, int fdt, const alto_mttkrp_plan &p) {
    h->tuned[mode][fdt][rank / 4] = p;
    h->has_tuned[mode][fdt][rank / 4] = true;
    const int rw = p.conflict == ALTO_CR_DIRECT ? direct_row_words(h, mode, rank, p) : 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[tune_key(h, mode, rank, fdt)] = {p, rw};
}

bool cached_tuned(const alto_tensor *h, int mode, int rank, int fdt, alto_mttkrp_plan *p, int *row_words) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(tune_key(h, mode, rank, fdt));
    if (it == g_tune_cache.end()) return false;
    *p = it->second.p;
    *row_words = it->second.row_words;
    return true;
}

// Whether a cached plan's LDS tables fit this tensor's mode and device.  A
// whole-mode plan must also keep the row width it was tuned with: on a
// longer mode FP64 rows can turn into FP32 rows added by compare-and-swap,
// which retry on skewed modes (3.4 ms against 0.9 ms for the table merge on
// a 1338-row mode given the plan tuned on a 1044-row mode of its class).
bool plan_fits(const alto_tensor *h, int mode, int rank, const alto_mttkrp_plan &p, int row_words) {
    const int rt = p.rank_tile > 0 ? p.rank_tile : rank;
    if (p.block_threads != 256 && p.block_threads != 512) return false;
    if (p.rank_tile < 0 || p.rank_tile % 4 || rank % rt) return false;
    if (p.conflict == ALTO_CR_DIRECT)
        return (size_t)h->info.dims[mode] * (rt + 1) * 4 <= direct_table_limit(h, p.block_threads) &&
               direct_row_words(h, mode, rank, p) == row_words;
    if (p.conflict == ALTO_CR_TILE || p.conflict == ALTO_CR_HOT)
        return p.table_slots >= 16 && tile_plan_fits(h, rt, p.table_slots, p.block_threads);
    return true;
}

// Accuracy policy for plans that add into the FP32 output with FP32 atomics.
// Every partial row a workgroup flushes is one rounded FP32 addition into
// its output entries, and an addition can lose up to half a unit in the last
// place of the entry's running sum: partials that arrive after the entry has
// grown large are rounded away ("swamping").  An entry that takes K additions
// is thus off by up to K 2^-25 of the sum of its terms' magnitudes.  On
// skewed tensors the heavy rows take one partial per tile (or per workgroup)
// plus one per table miss, and after a CP-ALS update the factor values make
// most of those partials small; measured on the 1e8-nonzero Zipf tensor after
// one sweep, FP32 atomics left entries at 2-9 times 1e-5 of that sum.  So
// FP32 is kept only where K is bounded by kF32MaxAdds (K 2^-25 < 1e-5): by
// the tile count for the LDS table merge, the workgroup count for the
// whole-mode table (at most one flush per workgroup), the nonzero count for
// register runs.  Otherwise the plan accumulates in FP64: eight per-XCD FP64
// copies for short modes under heavy contention (atomics of different XCDs
// never meet), else one FP64 buffer.  Both round once to FP32 at the end.
constexpr uint64_t kF32MaxAdds = 256;
constexpr uint64_t kXcdCopyBytes = uint64_t(1) << 30;
constexpr double kXcdReuse = 512.0;

void accuracy_policy(const alto_tensor *h, int mode, int rank, alto_mttkrp_plan *p) {
    if (p->accumulate != ALTO_ACC_F32) return;
    const uint64_t nnz = h->info.nnz;
    const uint64_t tiles = (nnz + p->tile_nnz - 1) / (uint64_t)std::max(1, p->tile_nnz);
    uint64_t adds = nnz;
    if (p->conflict == ALTO_CR_TILE) adds = tiles;
    else if (p->conflict == ALTO_CR_DIRECT) adds = std::min<uint64_t>(tiles, (uint64_t)device_cus(h->device) * 4);
    if (adds <= kF32MaxAdds) return;
    const double reuse = (double)nnz / (double)std::max<uint64_t>(1, h->info.dims[mode]);
    const uint64_t copies = h->info.dims[mode] * (uint64_t)rank * 8 * kXcdCopies;
    p->accumulate = (reuse >= kXcdReuse && copies <= kXcdCopyBytes) ? ALTO_ACC_XCD_F64 : ALTO_ACC_F64;
}

// The other FP64 form of a plan the policy moved to FP64 (the autotuner
// times both); false when there is none that fits.
bool alternate_f64(const alto_tensor *h, int mode, int rank, alto_mttkrp_plan *p) {
    if (p->accumulate == ALTO_ACC_XCD_F64) {
        p->accumulate = ALTO_ACC_F64;
        return true;
    }
    if (p->accumulate != ALTO_ACC_F64) return false;
    if (h->info.dims[mode] * (uint64_t)rank * 8 * kXcdCopies > kXcdCopyBytes) return false;
    p->accumulate = ALTO_ACC_XCD_F64;
    return true;
}

alto_status resolve_plan(const alto_tensor *h, int mode, int rank, int fdt, const alto_mttkrp_plan *in,
                         alto_mttkrp_plan *out) {
    alto_mttkrp_plan p = default_plan(h, mode, rank, fdt);
    const int ri = rank / 4;
    if (ri >= 0 && ri <= 32 && h->has_tuned[mode][fdt][ri]) {
        p = h->tuned[mode][fdt][ri];
    } else if (ri >= 0 && ri <= 32) {
        // a plan tuned on another tensor of the class is used only where it
        // fits this one (its mode may be longer than the tuned one's)
        alto_mttkrp_plan c;
        int rw = 0;
        if (cached_tuned(h, mode, rank, fdt, &c, &rw) && plan_fits(h, mode, rank, c, rw)) p = c;
    }
    if (in) {
        if (in->conflict) {
            p.conflict = in->conflict;
            p.rank_tile = 0;
        }
        if (in->rank_tile) p.rank_tile = in->rank_tile;
        if (in->tile_order) p.tile_order = in->tile_order;
        if (in->tile_nnz) p.tile_nnz = in->tile_nnz;
        if (in->block_threads) p.block_threads = in->block_threads;
        if (in->table_slots) p.table_slots = in->table_slots;
        if (in->accumulate) p.accumulate = in->accumulate;
    }
    if (p.accumulate < ALTO_ACC_F64 || p.accumulate > ALTO_ACC_XCD_F64) return fail(ALTO_ERR_ARG, "bad accumulate mode");
    // an accumulation the caller did not choose follows the accuracy policy
    if (!(in && in->accumulate)) accuracy_policy(h, mode, rank, &p);
    if (p.conflict != ALTO_CR_TILE && p.conflict != ALTO_CR_RUN && p.conflict != ALTO_CR_DIRECT &&
        p.conflict != ALTO_CR_HOT)
        return fail(ALTO_ERR_ARG, "bad conflict mode");
    if (p.conflict == ALTO_CR_HOT && h->info.nmodes > 5)
        return fail(ALTO_ERR_ARG, "hot-row merging supports tensors of up to 5 modes");
    if (p.tile_order < ALTO_ORDER_DEFAULT || p.tile_order > ALTO_ORDER_INTERLEAVED)
        return fail(ALTO_ERR_ARG, "bad tile order");
    if (p.rank_tile < 0 || p.rank_tile % 4 || (p.rank_tile > 0 && rank % p.rank_tile))
        return fail(ALTO_ERR_ARG, "rank_tile must be a multiple of 4 dividing rank");
    const int rt = p.rank_tile > 0 ? p.rank_tile : rank;
    if (p.block_threads != 256 && p.block_threads != 512) return fail(ALTO_ERR_ARG, "block_threads must be 256 or 512");
    if (p.conflict == ALTO_CR_DIRECT &&
        (size_t)h->info.dims[mode] * (rt + 1) * 4 > direct_table_limit(h, p.block_threads))
        return fail(ALTO_ERR_ARG, "mode too long to hold in LDS for this rank tile");
    if (p.tile_nnz < 1) return fail(ALTO_ERR_ARG, "tile_nnz must be positive");
    if (p.conflict == ALTO_CR_TILE || p.conflict == ALTO_CR_HOT) {
        if (p.table_slots < 16 || (p.table_slots & (p.table_slots - 1)))
            return fail(ALTO_ERR_ARG, "table_slots must be a power of two >= 16");
        // FP64 rows + keys + hit counts, the record staging and static LDS
        if (!tile_plan_fits(h, rt, p.table_slots, p.block_threads))
            return fail(ALTO_ERR_ARG, "LDS table too large for rank and block size");
    }
    *out = p;
    return ALTO_OK;
}

alto_status check_mttkrp_args(const alto_tensor *h, int mode, int rank, int fdt, const void *const *factors,
                              const float *out) {
    ALTO_CHECK_HANDLE(h);
    if (mode < 0 || mode >= h->info.nmodes) return fail(ALTO_ERR_ARG, "mode out of range");
    if (rank < 1 || rank > ALTO_MAX_RANK) return fail(ALTO_ERR_ARG, "rank must be in 1..128");
    if (fdt != ALTO_F32 && fdt != ALTO_BF16) return fail(ALTO_ERR_ARG, "bad factor dtype");
    if (!out) return fail(ALTO_ERR_ARG, "out is NULL");
    // rows of a multiple-of-4 rank are read and written 4 columns at a time;
    // other ranks go through padded copies and need element alignment only
    const bool vec = rank % 4 == 0;
    if (((uintptr_t)out & (vec ? 15 : 3)) != 0) return fail(ALTO_ERR_ARG, "out must be 16-byte aligned");
    if (!factors) return fail(ALTO_ERR_ARG, "factors is NULL");
    const uintptr_t al = vec ? (fdt == ALTO_F32 ? 15 : 7) : (fdt == ALTO_F32 ? 3 : 1);
    for (int m = 0; m < h->info.nmodes; m++) {
        if (m == mode) continue;
        if (!factors[m]) return fail(ALTO_ERR_ARG, "factors[" + std::to_string(m) + "] is NULL");
        if ((uintptr_t)factors[m] & al) return fail(ALTO_ERR_ARG, "factor rows must be 16-byte (8 for BF16) aligned");
    }
    return ALTO_OK;
}

namespace {
// dst (I x ldd) from src (I x lds): the first min(lds, ldd) columns, zeros after.
template <typename T>
__global__ void k_copy_cols(const T *__restrict__ src, int lds, T *__restrict__ dst, int ldd, uint64_t I) {
    const uint64_t n = I * (uint64_t)ldd;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const uint64_t i = t / (uint64_t)ldd;
        const int c = (int)(t - i * (uint64_t)ldd);
        dst[t] = c < lds ? src[i * (uint64_t)lds + c] : T(0);
    }
}
}  // namespace

void launch_copy_cols(const void *src, int lds, void *dst, int ldd, uint64_t I, int esize, hipStream_t s) {
    const unsigned g = grid_for(I * (uint64_t)ldd, 256, 16384);
    if (esize == 2)
        hipLaunchKernelGGL(k_copy_cols<uint16_t>, dim3(g), dim3(256), 0, s, (const uint16_t *)src, lds, (uint16_t *)dst,
                           ldd, I);
    else
        hipLaunchKernelGGL(k_copy_cols<float>, dim3(g), dim3(256), 0, s, (const float *)src, lds, (float *)dst, ldd, I);
}

alto_status pad_factors(alto_tensor *h, int rank, int fdt, const void *const *factors, int skip, void **fptr,
                        hipStream_t s) {
    const int R4 = padded_rank(rank);
    const int es = fdt == ALTO_BF16 ? 2 : 4;
    for (int m = 0; m < h->info.nmodes; m++) {
        fptr[m] = nullptr;
        if (m == skip) continue;
        if (!factors[m]) return fail(ALTO_ERR_ARG, "factors[" + std::to_string(m) + "] is NULL");
        alto_status st = ensure_ws(&h->ws_pad[m], &h->ws_pad_bytes[m], h->info.dims[m] * (size_t)R4 * es, s);
        if (st != ALTO_OK) return st;
        launch_copy_cols(factors[m], rank, h->ws_pad[m], R4, h->info.dims[m], es, s);
        fptr[m] = h->ws_pad[m];
    }
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

alto_status ensure_ws(void **p, size_t *have, size_t need, hipStream_t s) {
    if (*have >= need && *p) return ALTO_OK;
    if (*p) {
        // the old buffer returns to the cache behind the work already on s
        dev_free_after(*p, s);
        *p = nullptr;
        *have = 0;
    }
    if (dev_alloc(p, need) != hipSuccess) return fail(ALTO_ERR_OOM, "workspace allocation failed");
    *have = need;
    return ALTO_OK;
}

void fill_args(const alto_tensor *h, int mode, int rank, int fdt, const void *const *factors,
               const alto_mttkrp_plan &p, float *out32, double *out64, MttkrpArgs *a, int col0, int rank_tile) {
    memset(a, 0, sizeof(*a));
    a->lp = h->lp;
    int k = 0;
    for (int m = 0; m < h->info.nmodes; m++)
        if (m != mode) {
            a->last_other[k] = (uint32_t)(h->info.dims[m] - 1);
            a->fac_other[k++] = factors[m];
        }
    a->dim_out = (uint32_t)h->info.dims[mode];
    // 32-bit buffer offsets reach every factor row when each factor is below 2 GiB
    const int fbytes = fdt == ALTO_BF16 ? 2 : 4;
    a->buf32 = 1;
    k = 0;
    for (int m = 0; m < h->info.nmodes; m++) {
        if (m == mode) continue;
        const uint64_t bytes = h->info.dims[m] * (uint64_t)rank * fbytes;
        if (bytes >= (uint64_t(1) << 31)) a->buf32 = 0;
        a->fac_bytes[k++] = (uint32_t)(bytes < (uint64_t(1) << 31) ? bytes : 0);
    }
    a->keys = h->keys;
    a->vals = h->vals;
    a->out32 = out32;
    a->out64 = out64;
    a->nnz = h->info.nnz;
    uint64_t L = (h->info.nnz + p.tile_nnz - 1) / p.tile_nnz;
    if (L < 1) L = 1;
    a->ntiles = L;
    a->tq = h->info.nnz / L;
    a->tr = h->info.nnz % L;
    a->mode = mode;
    a->rank = rank_tile > 0 ? rank_tile : rank;
    a->ld = (uint32_t)rank;
    a->col0 = (uint32_t)col0;
    a->nmodes = h->info.nmodes;
    a->tile_merge = p.conflict == ALTO_CR_TILE ? 1 : p.conflict == ALTO_CR_DIRECT ? 2 : p.conflict == ALTO_CR_HOT ? 3 : 0;
    a->use64 = (p.accumulate == ALTO_ACC_F64 || p.accumulate == ALTO_ACC_XCD_F64) ? 1 : 0;
    a->copies = (p.accumulate == ALTO_ACC_XCD_F32 || p.accumulate == ALTO_ACC_XCD_F64) ? kXcdCopies : 1;
    a->copy_stride = h->info.dims[mode] * (uint64_t)rank;
    int l2 = 0;
    while ((1 << l2) < p.table_slots) l2++;
    a->slots_log2 = l2;
    a->rec = record_words(h->info.nmodes, h->info.index_words);
    a->interleave = p.tile_order == ALTO_ORDER_INTERLEAVED && p.conflict != ALTO_CR_HOT;
    a->lut = h->info.nmodes == 3 && h->info.index_words == 1;
    for (int m = 0; m < h->info.nmodes; m++)
        if (h->info.nbits[m] > 21) a->lut = 0;
    // whole-mode rows are FP64 when this rank tile fits so, else FP32
    a->tw = 2;
    if (a->tile_merge == 2 &&
        (size_t)h->info.dims[mode] * (a->rank + 1) * 8 > direct_table_limit(h, p.block_threads))
        a->tw = 1;
}

size_t lds_bytes(const MttkrpArgs &a, int threads) {
    const bool hashed = a.tile_merge == 1 || a.tile_merge == 3;
    const size_t S = hashed ? ((size_t)1 << a.slots_log2) : (a.tile_merge == 2 ? a.dim_out : 0);
    const size_t SK = hashed ? S : 0;
    const size_t TW = a.tile_merge == 2 ? (size_t)a.tw : 2;  // words per table element
    // the whole-mode table needs no outbox: all its rows are in LDS
    const size_t ob = a.tile_merge == 2 ? 0 : outbox_bytes(a.rank, threads);
    return ((2 * SK + TW * S * (a.rank + 1) + 3) & ~(size_t)3) * 4 + (size_t)threads * a.rec * 4 + ob;
}

// ---- optional per-launch timing with HIP events
namespace {
struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> pool;
};
Timing &timing() {
    static Timing *t = new Timing();
    return *t;
}
hipEvent_t take_event(Timing &t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}
void clear_pending(Timing &t) {
    for (auto &pr : t.pending) {
        (void)hipEventSynchronize(pr.second);
        t.pool.push_back(pr.first);
        t.pool.push_back(pr.second);
    }
    t.pending.clear();
}
}  // namespace

bool timing_begin(hipStream_t s, hipEvent_t *e0, hipEvent_t *e1) {
    Timing &t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.on) return false;
    *e0 = take_event(t);
    *e1 = take_event(t);
    if (!*e0 || !*e1) return false;
    (void)hipEventRecord(*e0, s);
    return true;
}

void timing_end(hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    Timing &t = timing();
    (void)hipEventRecord(e1, s);
    std::lock_guard<std::mutex> lk(t.mu);
    t.pending.push_back({e0, e1});
}

alto_status launch_mttkrp(const alto_tensor *h, int fdt, const MttkrpArgs &a, int threads, hipStream_t s) {
    const int lpn = lpn_for(a.rank);
    return launch_stretch_kernel(h, pick_single(lpn, fdt, h->info.index_words, a), a, threads, s);
}

alto_status launch_stretch_kernel(const alto_tensor *h, const void *kern, const MttkrpArgs &a, int threads,
                                  hipStream_t s) {
    const size_t lds = lds_bytes(a, threads);
    // never dispatch more LDS than a workgroup may hold
    alto_status lst = check_launch_lds(kern, lds, h->device);
    if (lst != ALTO_OK) return lst;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, lds) != hipSuccess || occ < 1) {
        (void)hipGetLastError();
        occ = 1;
    }
    const int cus = props(h->device).cus;
    uint64_t grid = (uint64_t)cus * occ;
    MttkrpArgs b = a;
    if (grid >= a.ntiles) {
        grid = a.ntiles;
        b.xcd_map = 0;
    } else {
        grid = grid / 8 * 8;
        b.xcd_map = 1;
    }
    if (grid < 1) grid = 1;
    void *args[] = {(void *)&b};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = timing_begin(s, &e0, &e1);
    ALTO_HIP(hipLaunchKernel(kern, dim3((unsigned)grid), dim3(threads), args, lds, s));
    if (timed) timing_end(s, e0, e1);
    return ALTO_OK;
}

alto_status run_mttkrp(alto_tensor *h, int mode, int rank, int fdt, const void *const *factors, float *out,
                       const alto_mttkrp_plan &p, hipStream_t s, void *acc_buf) {
    h->stream = s;
    const uint64_t nout = h->info.dims[mode] * (uint64_t)rank;
    const bool f64 = p.accumulate == ALTO_ACC_F64 || p.accumulate == ALTO_ACC_XCD_F64;
    const int copies = (p.accumulate == ALTO_ACC_XCD_F32 || p.accumulate == ALTO_ACC_XCD_F64) ? kXcdCopies : 1;
    const bool direct = p.accumulate == ALTO_ACC_F32;  // atomics straight into `out`
    const unsigned g = grid_for(nout * copies, 256, 16384);
    double *out64 = nullptr;
    float *acc32 = out;
    if (!direct) {
        // the accumulation buffer: the caller's (sized by the caller), else
        // handle workspace
        void *buf = acc_buf;
        if (!buf) {
            alto_status st = ensure_ws(&h->ws_acc, &h->ws_acc_bytes, nout * copies * (f64 ? 8 : 4), s);
            if (st != ALTO_OK) return st;
            buf = h->ws_acc;
        }
        if (f64) {
            out64 = (double *)buf;
            hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(256), 0, s, out64, nout * copies, 0.0);
        } else {
            acc32 = (float *)buf;
            hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(256), 0, s, acc32, nout * copies, 0.f);
        }
    } else {
        hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(256), 0, s, out, nout, 0.f);
    }
    ALTO_HIP(hipGetLastError());
    if (h->info.nnz > 0) {
        // one launch per rank tile (columns [c, c + rt) of factors and output)
        const int rt = p.rank_tile > 0 ? p.rank_tile : rank;
        for (int c = 0; c < rank; c += rt) {
            MttkrpArgs a;
            fill_args(h, mode, rank, fdt, factors, p, acc32, out64, &a, c, rt);
            alto_status st = launch_mttkrp(h, fdt, a, p.block_threads, s);
            if (st != ALTO_OK) return st;
        }
    }
    if (!direct) {
        const unsigned g1 = grid_for(nout, 256, 16384);
        if (f64) hipLaunchKernelGGL(k_sum_copies<double>, dim3(g1), dim3(256), 0, s, out64, copies, nout, out);
        else hipLaunchKernelGGL(k_sum_copies<float>, dim3(g1), dim3(256), 0, s, acc32, copies, nout, out);
        ALTO_HIP(hipGetLastError());
    }
    return ALTO_OK;
}

// ---- allocation-free MTTKRP with FP64 accumulation (alto_mttkrp_noalloc)
//
// Its accumulation buffer is this file-scope device array, which every GPU
// the library runs on holds until the process ends.  Host code never uses
// the array's name as an address: once per device, with that device
// current, its device address is looked up with hipGetSymbolAddress and kept;
// kernels receive that address.  Calls that overlap on one GPU share the
// array and race; every call clears what it uses first.
constexpr uint64_t kScratchDoubles = uint64_t(1) << 23;  // 64 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[64] = {};

alto_status scratch_for(int dev, double **out) {
    if (dev < 0 || dev >= 64) return fail(ALTO_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ALTO_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return ALTO_OK;
}
}  // namespace

}  // namespace alto

using namespace alto;

extern "C" {

alto_status alto_mttkrp_noalloc(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors,
                                float *out, const alto_mttkrp_plan *plan, void *stream) {
    alto_status st = check_mttkrp_args(h, mode, rank, fdt, factors, out);
    if (st != ALTO_OK) return st;
    if (rank % 4) return fail(ALTO_ERR_ARG, "alto_mttkrp_noalloc: rank must be a multiple of 4");
    if (plan && plan->accumulate != ALTO_ACC_DEFAULT && plan->accumulate != ALTO_ACC_F64)
        return fail(ALTO_ERR_ARG, "alto_mttkrp_noalloc accumulates in FP64 only");
    const uint64_t nout = h->info.dims[mode] * (uint64_t)rank;
    if (nout > kScratchDoubles)
        return fail(ALTO_ERR_ARG, "alto_mttkrp_noalloc: dims[mode] x rank = " + std::to_string(nout) +
                                      " exceeds the static scratch of " + std::to_string(kScratchDoubles) +
                                      " doubles");
    int dev = -1;
    ALTO_HIP(hipGetDevice(&dev));
    if (dev != h->device) return fail(ALTO_ERR_ARG, "the handle's device is not the current device");
    double *buf = nullptr;
    st = scratch_for(dev, &buf);
    if (st != ALTO_OK) return st;
    alto_mttkrp_plan p;
    st = resolve_plan(h, mode, rank, fdt, plan, &p);
    if (st != ALTO_OK) return st;
    p.accumulate = ALTO_ACC_F64;
    return run_mttkrp(h, mode, rank, fdt, factors, out, p, (hipStream_t)stream, buf);
}

alto_status alto_mttkrp_ex(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors, float *out,
                           const alto_mttkrp_plan *plan, void *stream) {
    alto_status st = check_mttkrp_args(h, mode, rank, fdt, factors, out);
    if (st != ALTO_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    alto_mttkrp_plan p;
    if (rank % 4 == 0) {
        st = resolve_plan(h, mode, rank, fdt, plan, &p);
        if (st != ALTO_OK) return st;
        return run_mttkrp(h, mode, rank, fdt, factors, out, p, s);
    }
    // zero-padded copies of the factors and the output at the next multiple of 4
    const int R4 = padded_rank(rank);
    st = resolve_plan(h, mode, R4, fdt, plan, &p);
    if (st != ALTO_OK) return st;
    void *pf[ALTO_MAX_MODES];
    st = pad_factors(h, rank, fdt, factors, mode, pf, s);
    if (st != ALTO_OK) return st;
    st = ensure_ws((void **)&h->ws_pad_out, &h->ws_pad_out_bytes, h->info.dims[mode] * (size_t)R4 * 4, s);
    if (st != ALTO_OK) return st;
    st = run_mttkrp(h, mode, R4, fdt, (const void *const *)pf, h->ws_pad_out, p, s);
    if (st != ALTO_OK) return st;
    launch_copy_cols(h->ws_pad_out, R4, out, rank, h->info.dims[mode], 4, s);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

alto_status alto_mttkrp(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors, float *out,
                        void *stream) {
    return alto_mttkrp_ex(h, mode, rank, fdt, factors, out, nullptr, stream);
}

alto_status alto_timing_enable(int on) {
    Timing &t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    clear_pending(t);
    t.on = on != 0;
    return ALTO_OK;
}

alto_status alto_timing_read(uint64_t *launches, double *total_ms) {
    if (!launches || !total_ms) return fail(ALTO_ERR_ARG, "NULL argument");
    Timing &t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    double tot = 0.0;
    for (auto &pr : t.pending) {
        float ms = 0.f;
        ALTO_HIP(hipEventSynchronize(pr.second));
        ALTO_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        tot += ms;
    }
    *launches = t.pending.size();
    *total_ms = tot;
    clear_pending(t);
    return ALTO_OK;
}

alto_status alto_release_cached_memory(void) {
    ALTO_HIP(hipDeviceSynchronize());
    release_cached();
    return ALTO_OK;
}

alto_status alto_mttkrp_get_plan(alto_handle h, int mode, int rank, alto_dtype fdt, alto_mttkrp_plan *out) {
    ALTO_CHECK_HANDLE(h);
    if (!out) return fail(ALTO_ERR_ARG, "out is NULL");
    if (mode < 0 || mode >= h->info.nmodes) return fail(ALTO_ERR_ARG, "mode out of range");
    if (rank < 1 || rank > ALTO_MAX_RANK) return fail(ALTO_ERR_ARG, "rank must be in 1..128");
    if (fdt != ALTO_F32 && fdt != ALTO_BF16) return fail(ALTO_ERR_ARG, "bad factor dtype");
    return resolve_plan(h, mode, padded_rank(rank), fdt, nullptr, out);
}

}  // extern "C"
