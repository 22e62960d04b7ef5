// CP-APR model update Phi over the ALTO line (Algorithm "alg:cp-apr-mu",
// Phi and Pi lines; Algorithm "fig:subproblem_algo"; Sec. "Adaptive Memory
// Management"): the MTTKRP machinery with a per-nonzero scale
// v / max(B(i_n, :) . krp, eps), the Khatri-Rao row krp either formed on
// the fly from the factors (ALTO-OTF) or read from a precomputed Pi
// (ALTO-PRE).  Conflict resolution as for MTTKRP (TILE / RUN / DIRECT),
// always over the whole rank: the dot product needs every column.
#include <string.h>

#include <string>

#include "memory.h"
#include "mttkrp_kernels.h"

namespace alto {
namespace {

constexpr int kPhiRec = 8;  // record words of the Phi kernels

const void *phi_kernel(int lpn, int words, bool pre) {
    if (words == 2) return pre ? phi_lpn<2, kOpPhiPre>(lpn) : phi_lpn<2, kOpPhi>(lpn);
    return pre ? phi_lpn<1, kOpPhiPre>(lpn) : phi_lpn<1, kOpPhi>(lpn);
}

alto_status check_phi_args(const alto_tensor *h, int mode, int rank, const void *const *factors, bool need_factors) {
    ALTO_CHECK_HANDLE(h);
    if (mode < 0 || mode >= h->info.nmodes) return fail(ALTO_ERR_ARG, "mode out of range");
    if (rank < 4 || rank > ALTO_MAX_RANK || rank % 4) return fail(ALTO_ERR_ARG, "Phi rank must be a multiple of 4 in 4..128");
    if (h->info.nmodes > 5) return fail(ALTO_ERR_ARG, "Phi supports tensors of up to 5 modes");
    if (need_factors) {
        if (!factors) return fail(ALTO_ERR_ARG, "factors is NULL");
        for (int m = 0; m < h->info.nmodes; m++) {
            if (m == mode) continue;
            if (!factors[m]) return fail(ALTO_ERR_ARG, "factors[" + std::to_string(m) + "] is NULL");
            if ((uintptr_t)factors[m] & 15) return fail(ALTO_ERR_ARG, "factors must be 16-byte aligned");
        }
    }
    return ALTO_OK;
}

// LDS of a Phi plan: table (TILE: keys, hits, FP64 rows; DIRECT: the mode's
// rows), 8-word records per thread and static arrays.
size_t phi_lds(const alto_tensor *h, int mode, int rank, const alto_mttkrp_plan &p, int tw) {
    size_t table = 0;
    if (p.conflict == ALTO_CR_TILE) table = (size_t)p.table_slots * (2 * (rank + 1) + 2) * 4;
    else if (p.conflict == ALTO_CR_DIRECT) table = (size_t)h->info.dims[mode] * (rank + 1) * 4 * tw;
    const size_t ob = p.conflict == ALTO_CR_DIRECT ? 0 : outbox_bytes(rank, p.block_threads);
    return table + (size_t)p.block_threads * kPhiRec * 4 + ob + static_lds_allowance();
}

// The MTTKRP plan of the mode, adapted to the Phi kernels: full rank in one
// pass, tables shrunk (or the conflict mode changed) until they fit.
alto_mttkrp_plan phi_plan(const alto_tensor *h, int mode, int rank, const alto_mttkrp_plan *in, int *tw) {
    alto_mttkrp_plan p;
    if (resolve_plan(h, mode, rank, ALTO_F32, in, &p) != ALTO_OK) {
        memset(&p, 0, sizeof(p));
        p.conflict = ALTO_CR_TILE;
        p.tile_nnz = 4096;
        p.block_threads = 256;
        p.table_slots = 256;
        p.accumulate = ALTO_ACC_F32;
    }
    p.rank_tile = 0;
    if (p.conflict == ALTO_CR_HOT) p.conflict = ALTO_CR_TILE;
    // Phi sums like MTTKRP: FP64 wherever the policy chose an FP64 form
    p.accumulate = (p.accumulate == ALTO_ACC_F64 || p.accumulate == ALTO_ACC_XCD_F64) ? ALTO_ACC_F64 : ALTO_ACC_F32;
    if (p.table_slots < 16) p.table_slots = 256;
    const size_t lim = device_lds(h->device);
    *tw = 2;
    if (p.conflict == ALTO_CR_DIRECT) {
        if (phi_lds(h, mode, rank, p, 2) > lim) *tw = 1;
        if (phi_lds(h, mode, rank, p, 1) > lim) p.conflict = ALTO_CR_TILE;
    }
    if (p.conflict == ALTO_CR_TILE) {
        while (p.table_slots > 16 && phi_lds(h, mode, rank, p, 2) > lim) p.table_slots /= 2;
        if (phi_lds(h, mode, rank, p, 2) > lim) p.conflict = ALTO_CR_RUN;
    }
    return p;
}

}  // namespace

alto_status run_phi(alto_tensor *h, int mode, int rank, const void *const *factors, const float *B, float eps,
                    const float *pi, float *phi, const alto_mttkrp_plan *in, hipStream_t s) {
    h->stream = s;
    int tw = 2;
    const alto_mttkrp_plan p = phi_plan(h, mode, rank, in, &tw);
    const uint64_t nout = h->info.dims[mode] * (uint64_t)rank;
    const bool f64 = p.accumulate == ALTO_ACC_F64;
    double *out64 = nullptr;
    const unsigned g = grid_for(nout, 256, 16384);
    if (f64) {
        alto_status st = ensure_ws(&h->ws_acc, &h->ws_acc_bytes, nout * 8, s);
        if (st != ALTO_OK) return st;
        out64 = (double *)h->ws_acc;
        hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(256), 0, s, out64, nout, 0.0);
    } else {
        hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(256), 0, s, phi, nout, 0.f);
    }
    ALTO_HIP(hipGetLastError());
    if (h->info.nnz > 0) {
        const void *nofac[ALTO_MAX_MODES] = {};
        MttkrpArgs a;
        fill_args(h, mode, rank, ALTO_F32, factors ? factors : nofac, p, phi, out64, &a, 0, rank);
        a.rec = kPhiRec;
        a.tw = p.conflict == ALTO_CR_DIRECT ? tw : 2;
        a.phi_B = B;
        a.phi_pi = pi;
        a.phi_eps = eps;
        alto_status st = launch_stretch_kernel(h, phi_kernel(lpn_for(rank), h->info.index_words, pi != nullptr), a,
                                               p.block_threads, s);
        if (st != ALTO_OK) return st;
    }
    if (f64) {
        hipLaunchKernelGGL(k_sum_copies<double>, dim3(g), dim3(256), 0, s, out64, 1, nout, phi);
        ALTO_HIP(hipGetLastError());
    }
    return ALTO_OK;
}

// ALTO-PRE when fiber reuse is low (the conflict-resolution rule's
// threshold) and the other modes' factor matrices are well beyond the
// on-chip cache (Sec. "Adaptive Memory Management").
bool prefer_pre(const alto_tensor *h, int mode, int rank) {
    const double reuse = (double)h->info.nnz / (double)h->info.dims[mode];
    uint64_t fbytes = 0;
    for (int m = 0; m < h->info.nmodes; m++)
        if (m != mode) fbytes += h->info.dims[m] * (uint64_t)rank * 4;
    return reuse <= 4.0 && fbytes > 2 * device_cache_bytes(h->device);
}

alto_status run_pi(alto_tensor *h, int mode, int rank, const float *const *factors, float *pi, hipStream_t s) {
    if (h->info.nnz == 0) return ALTO_OK;
    h->stream = s;
    alto_mttkrp_plan p;
    memset(&p, 0, sizeof(p));
    p.conflict = ALTO_CR_RUN;
    p.tile_nnz = 4096;
    p.block_threads = 256;
    p.accumulate = ALTO_ACC_F32;
    MttkrpArgs a;
    fill_args(h, mode, rank, ALTO_F32, (const void *const *)factors, p, nullptr, nullptr, &a, 0, rank);
    const int lpn = lpn_for(rank);
    const void *kern = h->info.index_words == 2 ? phi_pi_lpn<2>(lpn) : phi_pi_lpn<1>(lpn);
    const unsigned grid = grid_for(h->info.nnz * (uint64_t)lpn, 256, 16384);
    void *args[] = {(void *)&a, (void *)&pi};
    ALTO_HIP(hipLaunchKernel(kern, dim3(grid), dim3(256), args, 0, s));
    return ALTO_OK;
}

}  // namespace alto

using namespace alto;

extern "C" {

alto_status alto_cpapr_pi(alto_handle h, int mode, int rank, const float *const *factors, float *pi, void *stream) {
    alto_status st = check_phi_args(h, mode, rank, (const void *const *)factors, true);
    if (st != ALTO_OK) return st;
    if (!pi || ((uintptr_t)pi & 15)) return fail(ALTO_ERR_ARG, "pi must be a 16-byte aligned device pointer");
    return run_pi(h, mode, rank, factors, pi, (hipStream_t)stream);
}

alto_status alto_cpapr_prefer_pre(alto_handle h, int mode, int rank, int *pre) {
    ALTO_CHECK_HANDLE(h);
    if (!pre) return fail(ALTO_ERR_ARG, "pre is NULL");
    if (mode < 0 || mode >= h->info.nmodes) return fail(ALTO_ERR_ARG, "mode out of range");
    if (rank < 1) return fail(ALTO_ERR_ARG, "rank must be positive");
    *pre = prefer_pre(h, mode, rank) ? 1 : 0;
    return ALTO_OK;
}

alto_status alto_cpapr_phi(alto_handle h, int mode, int rank, const float *const *factors, const float *B, float eps,
                           const float *pi, float *phi, const alto_mttkrp_plan *plan, void *stream) {
    alto_status st = check_phi_args(h, mode, rank, (const void *const *)factors, pi == nullptr);
    if (st != ALTO_OK) return st;
    if (!B || ((uintptr_t)B & 15)) return fail(ALTO_ERR_ARG, "B must be a 16-byte aligned device pointer");
    if (!phi || ((uintptr_t)phi & 15)) return fail(ALTO_ERR_ARG, "phi must be a 16-byte aligned device pointer");
    if (pi && ((uintptr_t)pi & 15)) return fail(ALTO_ERR_ARG, "pi must be 16-byte aligned");
    if (pi && h->info.nnz >= (uint64_t(1) << 32)) return fail(ALTO_ERR_ARG, "ALTO-PRE needs nnz < 2^32");
    if (!(eps > 0.f)) return fail(ALTO_ERR_ARG, "eps must be positive");
    return run_phi(h, mode, rank, (const void *const *)factors, B, eps, pi, phi, plan, (hipStream_t)stream);
}

}  // extern "C"
