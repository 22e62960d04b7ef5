// CP-APR by multiplicative updates (Algorithm "alg:cp-apr-mu"): the outer
// and inner loops around the Phi (and Pi) kernels of phi.hip.  Per outer
// iteration k and mode n: B = (A^(n) + S) Lambda with the inadmissible-zero
// adjustment S; up to l_max inner iterations of Phi, the KKT check
// max|min(B, 1 - Phi)| < tau and B = B * Phi; then lambda = the column sums
// of B and A^(n) = B Lambda^-1.  The elementwise steps and the reductions
// are the small kernels below (FP32 B and Phi, FP64 lambda and reductions
// in a fixed order); the host reads the KKT value once per inner iteration.
#include <string.h>

#include <algorithm>
#include <string>
#include <utility>

#include "alto_internal.h"
#include "device_util.h"
#include "memory.h"
#include "mttkrp.h"

namespace alto {
namespace {

constexpr int kAprThreads = 256;
constexpr unsigned kAprBlocks = 512;  // partial results per reduction
constexpr uint64_t kAprPiBudget = uint64_t(32) << 30;  // Pi rows precomputed up to this size

// B = (A + S) Lambda, S = kappa where A < kappa_tol and the mode's previous
// Phi exceeds 1 (phi_prev null in the first outer iteration: S = 0).
__global__ __launch_bounds__(kAprThreads) void k_apr_prep(const float *__restrict__ A, uint64_t n, int R,
                                                          const double *__restrict__ lam,
                                                          const float *__restrict__ phi_prev, double kappa,
                                                          double kappa_tol, float *__restrict__ B) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t start = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t step = (uint32_t)(stride % (uint64_t)R);
    uint32_t c = (uint32_t)(start % (uint64_t)R);  // column of t, advanced without a division per element
    for (uint64_t t = start; t < n; t += stride) {
        const double a = A[t];
        const double s = (phi_prev && a < kappa_tol && phi_prev[t] > 1.f) ? kappa : 0.0;
        B[t] = (float)((a + s) * lam[c]);
        c += step;
        if (c >= (uint32_t)R) c -= (uint32_t)R;
    }
}

__device__ inline double block_max(double v, double *sm) {
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
        __syncthreads();
    }
    return sm[0];
}

// The KKT violation max|min(B, 1 - Phi)| (per block), and the next iterate
// B * Phi into Bn (used only when the check fails).
__global__ __launch_bounds__(kAprThreads) void k_apr_kkt(const float *__restrict__ B, const float *__restrict__ Phi,
                                                         uint64_t n, float *__restrict__ Bn,
                                                         double *__restrict__ partial) {
    __shared__ double sm[kAprThreads];
    double m = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const float b = B[t], p = Phi[t];
        m = fmax(m, fabs(fmin((double)b, 1.0 - (double)p)));
        Bn[t] = b * p;
    }
    m = block_max(m, sm);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(kAprThreads) void k_apr_max_final(const double *__restrict__ partial, unsigned P,
                                                               double *__restrict__ out) {
    __shared__ double sm[kAprThreads];
    double m = 0.0;
    for (unsigned i = threadIdx.x; i < P; i += blockDim.x) m = fmax(m, partial[i]);
    m = block_max(m, sm);
    if (threadIdx.x == 0) *out = m;
}

// Column sums of B (I x R): block b sums rows b, b + P, ... per column in
// FP64; threads take (row group, column) pairs.
__global__ __launch_bounds__(kAprThreads) void k_apr_colsum(const float *__restrict__ B, uint64_t I, int R,
                                                            double *__restrict__ partial) {
    __shared__ double sm[kAprThreads];
    const int groups = kAprThreads / R;  // rows handled at once
    const int g = threadIdx.x / R, c = threadIdx.x % R;
    double s = 0.0;
    if (g < groups)
        for (uint64_t i = (uint64_t)blockIdx.x * groups + g; i < I; i += (uint64_t)gridDim.x * groups)
            s += B[i * R + c];
    sm[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < R) {
        double t = 0.0;
        for (int k = 0; k < groups; k++) t += sm[k * R + threadIdx.x];
        partial[(uint64_t)blockIdx.x * R + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(kAprThreads) void k_apr_colsum_final(const double *__restrict__ partial, unsigned P,
                                                                  int R, double *__restrict__ lam) {
    for (int c = threadIdx.x; c < R; c += blockDim.x) {
        double t = 0.0;
        for (unsigned b = 0; b < P; b++) t += partial[(uint64_t)b * R + c];
        lam[c] = t;
    }
}

// A = B Lambda^-1; a zero column stays zero.
__global__ __launch_bounds__(kAprThreads) void k_apr_normalize(const float *__restrict__ B, uint64_t n, int R,
                                                               const double *__restrict__ lam, float *__restrict__ A) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t start = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t step = (uint32_t)(stride % (uint64_t)R);
    uint32_t c = (uint32_t)(start % (uint64_t)R);
    for (uint64_t t = start; t < n; t += stride) {
        const double l = lam[c];
        A[t] = l > 0.0 ? (float)((double)B[t] / l) : 0.f;
        c += step;
        if (c >= (uint32_t)R) c -= (uint32_t)R;
    }
}

unsigned blocks_for(uint64_t n) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(kAprBlocks, (n + kAprThreads - 1) / kAprThreads));
}

alto_status check_apr_args(const alto_tensor *h, int rank, float *const *factors, const double *lambda,
                           const alto_cpapr_params *p) {
    ALTO_CHECK_HANDLE(h);
    if (rank < 4 || rank > ALTO_MAX_RANK || rank % 4) return fail(ALTO_ERR_ARG, "CP-APR rank must be a multiple of 4 in 4..128");
    if (h->info.nmodes > 5) return fail(ALTO_ERR_ARG, "CP-APR supports tensors of up to 5 modes");
    if (!factors || !lambda || !p) return fail(ALTO_ERR_ARG, "factors, lambda and params must not be NULL");
    for (int m = 0; m < h->info.nmodes; m++) {
        if (!factors[m]) return fail(ALTO_ERR_ARG, "factors[" + std::to_string(m) + "] is NULL");
        if ((uintptr_t)factors[m] & 15) return fail(ALTO_ERR_ARG, "factors must be 16-byte aligned");
    }
    if (p->k_max < 1 || p->l_max < 1) return fail(ALTO_ERR_ARG, "k_max and l_max must be at least 1");
    if (p->pi_form < 0 || p->pi_form > 2) return fail(ALTO_ERR_ARG, "pi_form must be 0, 1 or 2");
    if (!(p->tau >= 0.0) || !(p->kappa >= 0.0) || !(p->kappa_tol >= 0.0) || !(p->eps > 0.f))
        return fail(ALTO_ERR_ARG, "tau, kappa, kappa_tol must be >= 0 and eps > 0");
    return ALTO_OK;
}

}  // namespace
}  // namespace alto

using namespace alto;

extern "C" {

alto_status alto_cpapr_mu(alto_handle h, int rank, float *const *factors, double *lambda,
                          const alto_cpapr_params *params, int *outer_done, int *inner_counts, int *converged,
                          void *stream) {
    alto_status st = check_apr_args(h, rank, factors, lambda, params);
    if (st != ALTO_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    const int N = h->info.nmodes;
    const int R = rank;
    uint64_t maxI = 1;
    for (int m = 0; m < N; m++) maxI = std::max<uint64_t>(maxI, h->info.dims[m]);
    for (int m = 0; m < N; m++) {
        st = ensure_ws((void **)&h->ws_apr_phi[m], &h->ws_apr_phi_bytes[m], h->info.dims[m] * (size_t)R * 4, s);
        if (st != ALTO_OK) return st;
    }
    st = ensure_ws((void **)&h->ws_apr_b, &h->ws_apr_b_bytes, 2 * maxI * (size_t)R * 4, s);
    if (st != ALTO_OK) return st;
    st = ensure_ws((void **)&h->ws_apr_red, &h->ws_apr_red_bytes, ((size_t)kAprBlocks * R + 8) * 8, s);
    if (st != ALTO_OK) return st;
    // where Pi rows are precomputed (see the header for the rule)
    const uint64_t pi_bytes = h->info.nnz * (uint64_t)R * 4;
    bool use_pre[ALTO_MAX_MODES] = {};
    bool any_pre = false;
    for (int m = 0; m < N; m++) {
        const bool rule = prefer_pre(h, m, R) ||
                          (N >= 4 && params->l_max >= 5 && pi_bytes <= kAprPiBudget);
        use_pre[m] = params->pi_form == 1 || (params->pi_form == 0 && rule);
        // the PRE kernel addresses Pi rows with a 32-bit index
        if (h->info.nnz >= (uint64_t(1) << 32)) use_pre[m] = false;
        any_pre = any_pre || use_pre[m];
    }
    if (any_pre) {
        st = ensure_ws((void **)&h->ws_apr_pi, &h->ws_apr_pi_bytes, pi_bytes, s);
        if (st != ALTO_OK) return st;
    }
    double *partial = h->ws_apr_red;
    double *d_kkt = h->ws_apr_red + (size_t)kAprBlocks * R;
    const alto_cpapr_params &p = *params;
    int k = 0, total_conv = 0;
    for (k = 1; k <= p.k_max; k++) {
        bool conv = true;
        for (int n = 0; n < N; n++) {
            const uint64_t I = h->info.dims[n];
            const uint64_t ne = I * (uint64_t)R;
            const unsigned g = blocks_for(ne);
            float *B = h->ws_apr_b, *Bn = h->ws_apr_b + maxI * (size_t)R;
            float *phi = h->ws_apr_phi[n];
            hipLaunchKernelGGL(k_apr_prep, dim3(g), dim3(kAprThreads), 0, s, factors[n], ne, R, lambda,
                               k > 1 ? phi : nullptr, p.kappa, p.kappa_tol, B);
            ALTO_HIP(hipGetLastError());
            const bool pre = use_pre[n];
            if (pre) {
                st = run_pi(h, n, R, (const float *const *)factors, h->ws_apr_pi, s);
                if (st != ALTO_OK) return st;
            }
            int runs = 0;
            for (int l = 0; l < p.l_max; l++) {
                st = run_phi(h, n, R, (const void *const *)factors, B, p.eps, pre ? h->ws_apr_pi : nullptr, phi,
                             nullptr, s);
                if (st != ALTO_OK) return st;
                runs++;
                hipLaunchKernelGGL(k_apr_kkt, dim3(g), dim3(kAprThreads), 0, s, B, phi, ne, Bn, partial);
                hipLaunchKernelGGL(k_apr_max_final, dim3(1), dim3(kAprThreads), 0, s, partial, g, d_kkt);
                ALTO_HIP(hipGetLastError());
                double kkt = 0.0;
                ALTO_HIP(hipMemcpyAsync(&kkt, d_kkt, sizeof(double), hipMemcpyDeviceToHost, s));
                ALTO_HIP(hipStreamSynchronize(s));
                if (kkt < p.tau) break;
                conv = false;
                std::swap(B, Bn);  // B = B * Phi
            }
            if (inner_counts) inner_counts[(size_t)(k - 1) * N + n] = runs;
            const unsigned gc = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(kAprBlocks, I));
            hipLaunchKernelGGL(k_apr_colsum, dim3(gc), dim3(kAprThreads), 0, s, B, I, R, partial);
            hipLaunchKernelGGL(k_apr_colsum_final, dim3(1), dim3(kAprThreads), 0, s, partial, gc, R, lambda);
            hipLaunchKernelGGL(k_apr_normalize, dim3(g), dim3(kAprThreads), 0, s, B, ne, R, lambda, factors[n]);
            ALTO_HIP(hipGetLastError());
        }
        if (conv) {
            total_conv = 1;
            break;
        }
    }
    if (outer_done) *outer_done = std::min(k, p.k_max);
    if (converged) *converged = total_conv;
    return ALTO_OK;
}

}  // extern "C"
