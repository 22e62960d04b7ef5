// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "alto.h"

namespace alto {

constexpr uint32_t kHandleMagic = 0xA170A170u;
constexpr uint32_t kEmptyRow = 0xFFFFFFFFu;

// Bit extraction / deposit tables of one mode for one 64-bit index word.
// `mask` selects the word's bits that belong to the mode; mv[i] are the
// move masks of the parallel-suffix compress (Hacker's Delight, 2nd ed.,
// Sec. 7-4, "compress" with a constant mask): bit groups selected by mv[i]
// move right by 2^i in step i.  Deposit runs the same steps backwards.
struct WordMasks {
    uint64_t mask;
    uint64_t mv[6];
};

struct ModeMasks {
    WordMasks w[2];
    int lo_bits;  // bits of the mode held in word 0
    int pad;
};

// Everything a kernel needs to (de)linearize an index: passed by value in
// kernel arguments so that the masks live in scalar registers.
struct LinePlan {
    ModeMasks mode[ALTO_MAX_MODES];
    int nmodes;
    int words;
};

// All six steps run unconditionally: a zero move mask makes a step a no-op,
// and a branch per step would cost more scalar work than the step itself.
__host__ __device__ inline uint64_t compress_word(uint64_t x, const WordMasks &m) {
    x &= m.mask;
#pragma unroll
    for (int i = 0; i < 6; i++) {
        const uint64_t t = x & m.mv[i];
        x = (x ^ t) | (t >> (1u << i));
    }
    return x;
}

__host__ __device__ inline uint64_t deposit_word(uint64_t x, const WordMasks &m) {
#pragma unroll
    for (int i = 5; i >= 0; i--) {
        const uint64_t mv = m.mv[i];
        if (mv) x = (x & ~mv) | ((x << (1u << i)) & mv);
    }
    return x & m.mask;
}

// Coordinate of mode n from an index held in (lo, hi).
template <int WORDS>
__host__ __device__ inline uint32_t extract_mode(const ModeMasks &mm, uint64_t lo, uint64_t hi) {
    uint64_t c = compress_word(lo, mm.w[0]);
    if (WORDS == 2) c |= compress_word(hi, mm.w[1]) << mm.lo_bits;
    return (uint32_t)c;
}

// Host planner (plan.cpp).
alto_status make_plan(int nmodes, const uint64_t *dims, alto_info_t *info, LinePlan *lp);

// Thread-local error text.
alto_status fail(alto_status st, const std::string &msg);

}  // namespace alto

// Handle: owns the ordered ALTO tensor and all workspace.
struct alto_tensor {
    uint32_t magic;
    int device;
    alto_info_t info;
    alto::LinePlan lp;
    hipStream_t stream;  // stream of the last call that enqueued work for the handle
    uint64_t *keys;  // nnz * words, ordered by ALTO index
    float *vals;     // nnz
    // workspace (grown on demand)
    void *ws_acc;          // FP64 accumulation rows
    size_t ws_acc_bytes;
    void *ws_sweep;        // CP-ALS: Grams, partials, solve
    size_t ws_sweep_bytes;
    float *ws_m;           // CP-ALS: MTTKRP output buffer
    size_t ws_m_bytes;
    uint16_t *ws_bf16[ALTO_MAX_MODES];  // BF16 shadows of the factors
    size_t ws_bf16_bytes[ALTO_MAX_MODES];
    uint32_t *ws_flags;    // CP-ALS status flags (device)
    // ranks that are not a multiple of 4 run on zero-padded copies
    void *ws_pad[ALTO_MAX_MODES];  // factors with rank rounded up to a multiple of 4
    size_t ws_pad_bytes[ALTO_MAX_MODES];
    float *ws_pad_out;             // MTTKRP output of the padded rank
    size_t ws_pad_out_bytes;
    double *ws_lampad;             // lambda of the padded rank
    size_t ws_lampad_bytes;
    double *ws_fit;        // fit: [0] = ||X||^2 of the summed tensor, [1] = last fit (device)
    size_t ws_fit_bytes;
    bool xnorm_ready;      // ws_fit[0] holds ||X||^2
    // CP-APR: each mode's last Phi, the B iterates, reductions, Pi rows
    float *ws_apr_phi[ALTO_MAX_MODES];
    size_t ws_apr_phi_bytes[ALTO_MAX_MODES];
    float *ws_apr_b;
    size_t ws_apr_b_bytes;
    double *ws_apr_red;
    size_t ws_apr_red_bytes;
    float *ws_apr_pi;
    size_t ws_apr_pi_bytes;
    // per (mode, rank, dtype) tuned plans
    alto_mttkrp_plan tuned[ALTO_MAX_MODES][2][33];
    bool has_tuned[ALTO_MAX_MODES][2][33];
};

#define ALTO_HIP(call)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return alto::fail(ALTO_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_));      \
    } while (0)

#define ALTO_CHECK_HANDLE(h)                                                                        \
    do {                                                                                            \
        if (!(h) || (h)->magic != alto::kHandleMagic) return alto::fail(ALTO_ERR_STATE, "invalid alto handle"); \
    } while (0)
