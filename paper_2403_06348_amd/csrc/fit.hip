// Fit of a CP model and the CP-ALS driver (Algorithm "alg:cp-als": sweeps
// repeat until the fit ceases to improve).
//
// fit = 1 - ||X - Xhat||_F / ||X||_F for Xhat = sum_r lambda_r a_r^(0) o ...
// o a_r^(N-1), from the expansion
//   ||X - Xhat||^2 = ||X||^2 + lambda^T (*_m A^(m)T A^(m)) lambda
//                    - 2 sum_r lambda_r <M(:, r), A^(N-1)(:, r)>,
// where M is the MTTKRP of the last mode with the other factors.  After a
// sweep every term is already on the GPU: the sweep's Grams, the last
// mode's MTTKRP and lambda.  ||X||^2 is that of the tensor the nonzeros add
// up to: duplicate coordinates have equal ALTO indices, so they are
// neighbours on the ordered line and ||X||^2 is the sum over runs of equal
// indices of (sum of the run's values)^2.  It is computed once per handle
// by a three-level segmented reduction over the line:
//   level 1: each thread summarizes a chunk of kXnChunk nonzeros (its first
//            and last run's index and partial sum, the squared sums of the
//            runs strictly inside it, whether it is one run);
//   level 2: a workgroup combines its chunks' summaries the same way into a
//            summary of its kXnBlock nonzeros;
//   level 3: one workgroup combines the workgroup summaries.
// A run that crosses summaries is added up by the summary it starts in,
// walking forward over the summaries it covers.  FP64 throughout, fixed
// summation order: the result is deterministic.
#include <math.h>
#include <string.h>

#include <string>

#include "alto_internal.h"
#include "device_util.h"
#include "memory.h"
#include "mttkrp.h"

namespace alto {
namespace {

constexpr int kFitThreads = 256;
constexpr int kXnChunk = 64;                          // nonzeros per thread
constexpr int kXnBlock = kFitThreads * kXnChunk;      // nonzeros per workgroup

// Summary of a stretch of the ordered line.
struct RunSummary {
    uint64_t hk[2], tk[2];  // index of the first and of the last run
    double hs, ts;          // partial sums of the first and last run inside the stretch
    double inner;           // squared sums of the runs strictly inside
    int single;             // the stretch is one run (first run == last run)
    int empty;
};

__device__ inline bool key_eq(const uint64_t *a, const uint64_t *b) { return a[0] == b[0] && a[1] == b[1]; }

// Walk forward from summary c over the summaries its run `key` continues
// into, adding their first-run sums; *end is set when the walk runs past
// the last summary (the run reaches the end of the range).
__device__ inline double walk(const RunSummary *s, int n, int c, const uint64_t *key, double total, bool *end) {
    *end = false;
    for (int j = c + 1;; j++) {
        if (j >= n || s[j].empty) {
            *end = true;
            return total;
        }
        if (!key_eq(s[j].hk, key)) return total;
        total += s[j].hs;
        if (!s[j].single) return total;
    }
}

// Combine summaries s[0..n) (in order) into a summary of their whole range.
// Every thread of the block calls it; the result is valid in thread 0.
// Runs that start in summary c > 0 and end inside the range are squared
// into `inner`; the range's first and last runs stay open.
__device__ void combine(const RunSummary *s, int n, RunSummary *out, double *red) {
    const int tid = threadIdx.x;
    __shared__ RunSummary res;
    if (tid == 0) {
        res.empty = n == 0 || s[0].empty;
        res.single = 0;
    }
    __syncthreads();
    double contrib = 0.0;
    for (int c = tid; c < n; c += kFitThreads) {
        if (s[c].empty) continue;
        contrib += s[c].inner;
        bool end = false;
        if (c == 0) {
            const double total = s[0].single ? walk(s, n, 0, s[0].hk, s[0].hs, &end) : s[0].hs;
            res.hk[0] = s[0].hk[0];
            res.hk[1] = s[0].hk[1];
            res.hs = total;
            if (end) {
                res.single = 1;
                res.tk[0] = s[0].hk[0];
                res.tk[1] = s[0].hk[1];
                res.ts = total;
            }
        } else if (!key_eq(s[c].hk, s[c - 1].tk)) {
            // the first run starts here
            const double total = s[c].single ? walk(s, n, c, s[c].hk, s[c].hs, &end) : s[c].hs;
            if (end) {
                res.tk[0] = s[c].hk[0];
                res.tk[1] = s[c].hk[1];
                res.ts = total;
            } else {
                contrib += total * total;
            }
        }
        if (!s[c].single) {
            const double total = walk(s, n, c, s[c].tk, s[c].ts, &end);
            if (end) {
                res.tk[0] = s[c].tk[0];
                res.tk[1] = s[c].tk[1];
                res.ts = total;
            } else {
                contrib += total * total;
            }
        }
    }
    // fixed-order block sum
    red[tid] = contrib;
    __syncthreads();
    for (int w = kFitThreads / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        res.inner = red[0];
        *out = res;
    }
    __syncthreads();
}

// Levels 1 and 2: workgroup b summarizes nonzeros [b*kXnBlock, ...).
template <int WORDS>
__global__ __launch_bounds__(kFitThreads) void k_xn_blocks(const uint64_t *__restrict__ keys,
                                                           const float *__restrict__ vals, uint64_t nnz,
                                                           RunSummary *__restrict__ out) {
    __shared__ RunSummary s[kFitThreads];
    __shared__ double red[kFitThreads];
    const int tid = threadIdx.x;
    const uint64_t x0 = (uint64_t)blockIdx.x * kXnBlock + (uint64_t)tid * kXnChunk;
    const uint64_t x1 = x0 + kXnChunk < nnz ? x0 + kXnChunk : nnz;
    RunSummary m;
    m.empty = 1;
    m.single = 1;
    m.inner = 0.0;
    m.hs = m.ts = 0.0;
    m.hk[0] = m.hk[1] = m.tk[0] = m.tk[1] = 0;
    uint64_t ck[2] = {0, 0};
    double sum = 0.0;
    int nruns = 0;
    for (uint64_t x = x0; x < x1; x++) {
        const uint64_t k[2] = {keys[x * WORDS], WORDS == 2 ? keys[x * WORDS + 1] : 0};
        const double v = (double)vals[x];
        if (nruns == 0) {
            m.hk[0] = k[0];
            m.hk[1] = k[1];
            ck[0] = k[0];
            ck[1] = k[1];
            sum = v;
            nruns = 1;
        } else if (k[0] == ck[0] && k[1] == ck[1]) {
            sum += v;
        } else {
            if (nruns == 1) m.hs = sum;
            else m.inner += sum * sum;
            ck[0] = k[0];
            ck[1] = k[1];
            sum = v;
            nruns++;
        }
    }
    if (nruns > 0) {
        m.empty = 0;
        m.tk[0] = ck[0];
        m.tk[1] = ck[1];
        m.ts = sum;
        if (nruns == 1) m.hs = sum;
        else m.single = 0;
    }
    s[tid] = m;
    __syncthreads();
    combine(s, kFitThreads, out + blockIdx.x, red);
}

// Level 3: one workgroup combines the nb workgroup summaries; the range's
// first and last runs close at the ends of the line.
__global__ __launch_bounds__(kFitThreads) void k_xn_final(const RunSummary *__restrict__ blocks, int nb,
                                                          double *__restrict__ xnorm2) {
    __shared__ double red[kFitThreads];
    __shared__ RunSummary all;
    combine(blocks, nb, &all, red);
    if (threadIdx.x == 0) {
        double r = 0.0;
        if (!all.empty) {
            r = all.inner + all.hs * all.hs;
            if (!all.single) r += all.ts * all.ts;
        }
        *xnorm2 = r;
    }
}

// Partial column dot products sum_i M[i, r] A[i, r] over the row range of
// workgroup b, FP64, written to part[b * R + r].
__global__ __launch_bounds__(kFitThreads) void k_fit_dot(const float *__restrict__ M, const float *__restrict__ A,
                                                         uint64_t I, int R, double *__restrict__ part) {
    __shared__ double red[kFitThreads];
    const int tid = threadIdx.x;
    const int per = kFitThreads / R;  // threads per column
    const int r = tid % R, k = tid / R;
    const uint64_t rows = (I + gridDim.x - 1) / gridDim.x;
    const uint64_t i0 = (uint64_t)blockIdx.x * rows;
    const uint64_t i1 = i0 + rows < I ? i0 + rows : I;
    double acc = 0.0;
    if (k < per)
        for (uint64_t i = i0 + k; i < i1; i += per) acc += (double)M[i * R + r] * (double)A[i * R + r];
    red[tid] = acc;
    __syncthreads();
    if (tid < R) {
        double s = 0.0;
        for (int j = 0; j < per; j++) s += red[j * R + tid];
        part[(uint64_t)blockIdx.x * R + tid] = s;
    }
}

// fit = 1 - sqrt(max(||X||^2 + lam^T V lam - 2 sum_r lam_r dot_r, 0)) / ||X||,
// V = Hadamard product of the N Grams.
__global__ __launch_bounds__(kFitThreads) void k_fit_final(const double *__restrict__ part, int P, int R, int N,
                                                           const double *__restrict__ grams,
                                                           const double *__restrict__ lam,
                                                           const double *__restrict__ xnorm2, double *__restrict__ fit) {
    __shared__ double red[kFitThreads];
    const int tid = threadIdx.x;
    double acc = 0.0;
    // lam^T V lam over the R x R entries
    for (int e = tid; e < R * R; e += kFitThreads) {
        const int a = e / R, b = e % R;
        double v = lam[a] * lam[b];
        for (int m = 0; m < N; m++) v *= grams[(size_t)m * R * R + e];
        acc += v;
    }
    // - 2 sum_r lam_r dot_r
    for (int r = tid; r < R; r += kFitThreads) {
        double d = 0.0;
        for (int b = 0; b < P; b++) d += part[(size_t)b * R + r];
        acc -= 2.0 * lam[r] * d;
    }
    red[tid] = acc;
    __syncthreads();
    for (int w = kFitThreads / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        const double xx = *xnorm2;
        const double r2 = fmax(xx + red[0], 0.0);
        *fit = xx > 0.0 ? 1.0 - sqrt(r2) / sqrt(xx) : 0.0;
    }
}

constexpr int kFitSlots = 2;  // ws_fit: [0] = ||X||^2, [1] = last fit

}  // namespace

// ||X||^2 of the handle's tensor into h->ws_fit[0], once per handle.
alto_status ensure_xnorm2(alto_tensor *h, hipStream_t s) {
    h->stream = s;
    size_t have = h->ws_fit_bytes;
    alto_status st = ensure_ws((void **)&h->ws_fit, &have, kFitSlots * sizeof(double), s);
    if (st != ALTO_OK) return st;
    h->ws_fit_bytes = have;
    if (h->xnorm_ready) return ALTO_OK;
    const uint64_t nnz = h->info.nnz;
    const uint64_t nb = (nnz + kXnBlock - 1) / kXnBlock;
    if (nb > (uint64_t)1 << 30) return fail(ALTO_ERR_ARG, "tensor too large for the norm reduction");
    RunSummary *sums = nullptr;
    if (nb > 0) {
        if (dev_alloc((void **)&sums, nb * sizeof(RunSummary)) != hipSuccess)
            return fail(ALTO_ERR_OOM, "norm reduction scratch allocation failed");
        if (h->info.index_words == 2)
            hipLaunchKernelGGL(k_xn_blocks<2>, dim3((unsigned)nb), dim3(kFitThreads), 0, s, h->keys, h->vals, nnz, sums);
        else
            hipLaunchKernelGGL(k_xn_blocks<1>, dim3((unsigned)nb), dim3(kFitThreads), 0, s, h->keys, h->vals, nnz, sums);
    }
    hipLaunchKernelGGL(k_xn_final, dim3(1), dim3(kFitThreads), 0, s, sums, (int)nb, h->ws_fit);
    const hipError_t e = hipGetLastError();
    if (sums) {
        // the scratch is returned to the cache once the reduction has run
        const hipError_t e2 = hipStreamSynchronize(s);
        dev_free(sums);
        if (e2 != hipSuccess) return fail(ALTO_ERR_HIP, std::string("norm reduction: ") + hipGetErrorString(e2));
    }
    if (e != hipSuccess) return fail(ALTO_ERR_HIP, std::string("norm reduction launch: ") + hipGetErrorString(e));
    h->xnorm_ready = true;
    return ALTO_OK;
}

// Fit of the model held in the sweep workspace (Grams of every factor, the
// last mode's MTTKRP in ws_m) with last factor A_last and weights lam, into
// the device double *fit.
alto_status launch_fit(alto_tensor *h, int rank, const float *A_last, const double *lam, double *fit, hipStream_t s) {
    const int N = h->info.nmodes;
    const size_t rr = (size_t)rank * rank;
    const double *grams = (const double *)h->ws_sweep;
    double *part = (double *)h->ws_sweep + N * rr + rr;  // the sweep's partial-Gram area
    const uint64_t I = h->info.dims[N - 1];
    unsigned P = (unsigned)((I + 1023) / 1024);
    if (P > kSweepPartials) P = kSweepPartials;
    if (P < 1) P = 1;
    hipLaunchKernelGGL(k_fit_dot, dim3(P), dim3(kFitThreads), 0, s, h->ws_m, A_last, I, rank, part);
    hipLaunchKernelGGL(k_fit_final, dim3(1), dim3(kFitThreads), 0, s, part, (int)P, rank, N, grams, lam,
                       h->ws_fit, fit);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

}  // namespace alto

using namespace alto;

extern "C" {

alto_status alto_cp_fit(alto_handle h, int rank, alto_dtype fdt, float *const *factors, const double *lambda,
                        double *fit, void *stream) {
    ALTO_CHECK_HANDLE(h);
    if (!fit) return fail(ALTO_ERR_ARG, "fit is NULL");
    if (!factors || !lambda) return fail(ALTO_ERR_ARG, "factors/lambda is NULL");
    if (rank < 1 || rank > 64) return fail(ALTO_ERR_ARG, "rank must be in 1..64");
    hipStream_t s = (hipStream_t)stream;
    alto_status st = ALTO_OK;
    void *pf[ALTO_MAX_MODES];
    if (rank % 4) {
        // zero-padded copies of the factors and of lambda
        const int R4 = padded_rank(rank);
        st = pad_factors(h, rank, ALTO_F32, (const void *const *)factors, -1, pf, s);
        if (st != ALTO_OK) return st;
        st = ensure_ws((void **)&h->ws_lampad, &h->ws_lampad_bytes, (size_t)R4 * sizeof(double), s);
        if (st != ALTO_OK) return st;
        hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, s, h->ws_lampad, (uint64_t)R4, 0.0);
        ALTO_HIP(hipMemcpyAsync(h->ws_lampad, lambda, (size_t)rank * sizeof(double), hipMemcpyDeviceToDevice, s));
        factors = (float *const *)pf;
        lambda = h->ws_lampad;
        rank = R4;
    }
    // Grams of every factor (and BF16 shadows) into the sweep workspace
    st = sweep_begin(h, rank, fdt, factors, lambda, s);
    if (st != ALTO_OK) return st;
    st = ensure_xnorm2(h, s);
    if (st != ALTO_OK) return st;
    const int N = h->info.nmodes;
    const void *fptr[ALTO_MAX_MODES];
    sweep_factor_ptrs(h, fdt, factors, fptr);
    alto_mttkrp_plan p;
    st = resolve_plan(h, N - 1, rank, fdt, nullptr, &p);
    if (st != ALTO_OK) return st;
    st = run_mttkrp(h, N - 1, rank, fdt, fptr, h->ws_m, p, s);
    if (st != ALTO_OK) return st;
    st = launch_fit(h, rank, factors[N - 1], lambda, h->ws_fit + 1, s);
    if (st != ALTO_OK) return st;
    ALTO_HIP(hipMemcpyAsync(fit, h->ws_fit + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    ALTO_HIP(hipStreamSynchronize(s));
    return ALTO_OK;
}

alto_status alto_tensor_norm2(alto_handle h, double *norm2, void *stream) {
    ALTO_CHECK_HANDLE(h);
    if (!norm2) return fail(ALTO_ERR_ARG, "norm2 is NULL");
    hipStream_t s = (hipStream_t)stream;
    alto_status st = ensure_xnorm2(h, s);
    if (st != ALTO_OK) return st;
    ALTO_HIP(hipMemcpyAsync(norm2, h->ws_fit, sizeof(double), hipMemcpyDeviceToHost, s));
    ALTO_HIP(hipStreamSynchronize(s));
    return ALTO_OK;
}

alto_status cpd_als(alto_handle h, int rank, alto_dtype fdt, float *const *factors, double *lambda, int max_sweeps,
                    double tol, double *fits, int *sweeps_done, void *stream) {
    ALTO_CHECK_HANDLE(h);
    if (max_sweeps < 1) return fail(ALTO_ERR_ARG, "max_sweeps must be >= 1");
    if (!(tol >= 0.0)) return fail(ALTO_ERR_ARG, "tol must be >= 0");
    if (!factors || !lambda) return fail(ALTO_ERR_ARG, "factors/lambda is NULL");
    if (rank < 1 || rank > 64) return fail(ALTO_ERR_ARG, "rank must be in 1..64");
    hipStream_t s = (hipStream_t)stream;
    if (sweeps_done) *sweeps_done = 0;
    const int N = h->info.nmodes;
    // a rank that is not a multiple of 4 runs on zero-padded copies, copied
    // back at the end
    const int R4 = padded_rank(rank);
    float *const *F = factors;
    double *lam = lambda;
    void *pf[ALTO_MAX_MODES];
    if (R4 != rank) {
        alto_status st = pad_factors(h, rank, ALTO_F32, (const void *const *)factors, -1, pf, s);
        if (st != ALTO_OK) return st;
        st = ensure_ws((void **)&h->ws_lampad, &h->ws_lampad_bytes, (size_t)R4 * sizeof(double), s);
        if (st != ALTO_OK) return st;
        F = (float *const *)pf;
        lam = h->ws_lampad;
    }
    double prev = 0.0;
    bool fallback = false;
    for (int k = 0; k < max_sweeps; k++) {
        alto_status st = sweep_run(h, R4, rank, fdt, F, lam, s);
        if (st != ALTO_OK) return st;
        if (k == 0) {
            st = ensure_xnorm2(h, s);
            if (st != ALTO_OK) return st;
        }
        st = launch_fit(h, R4, F[N - 1], lam, h->ws_fit + 1, s);
        if (st != ALTO_OK) return st;
        if (R4 != rank) {
            for (int m = 0; m < N; m++) launch_copy_cols(F[m], R4, factors[m], rank, h->info.dims[m], 4, s);
            ALTO_HIP(hipMemcpyAsync(lambda, lam, (size_t)rank * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        double f = 0.0;
        uint32_t flags = 0;
        ALTO_HIP(hipMemcpyAsync(&f, h->ws_fit + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        ALTO_HIP(hipMemcpyAsync(&flags, h->ws_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        ALTO_HIP(hipStreamSynchronize(s));
        if (flags) fallback = true;
        if (fits) fits[k] = f;
        if (sweeps_done) *sweeps_done = k + 1;
        if (k > 0 && fabs(f - prev) < tol) break;
        prev = f;
    }
    if (fallback) {
        fail(ALTO_ERR_NOT_SPD, "the pseudo-inverse was used in at least one mode update");
        return ALTO_ERR_NOT_SPD;
    }
    return ALTO_OK;
}

}  // extern "C"
