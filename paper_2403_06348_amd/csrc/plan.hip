// Host planner: bit layout of the ALTO index and the extraction tables.
//
// The layout follows Sec. "ALTO Tensor Generation" and Eq. 1 of the paper:
// mode n receives ceil(log2 I_n) bits (none when I_n = 1); the index is made
// of bit groups, group l holding bit l of every mode that has more than l
// bits, with the modes of a group ordered by increasing length (ties by mode
// number) so that the shortest mode takes the lowest position of the group
// and the most significant bits split the longest mode first.
#include <string.h>

#include <algorithm>
#include <string>

#include "alto_internal.h"

namespace alto {

static thread_local std::string g_last_error = "no error";

alto_status fail(alto_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

// Move masks of the parallel-suffix compress for a constant mask
// (Hacker's Delight, 2nd ed., Sec. 7-4).
static void move_masks(uint64_t m, uint64_t mv[6]) {
    uint64_t mk = ~m << 1;  // ones where a zero of m lies to the right
    for (int i = 0; i < 6; i++) {
        uint64_t mp = mk ^ (mk << 1);  // parallel suffix (prefix xor from the right)
        mp ^= mp << 2;
        mp ^= mp << 4;
        mp ^= mp << 8;
        mp ^= mp << 16;
        mp ^= mp << 32;
        const uint64_t v = mp & m;  // bits that move by 2^i in this step
        m = (m ^ v) | (v >> (1u << i));
        mk &= ~mp;
        mv[i] = v;
    }
}

static int ceil_log2(uint64_t d) {
    int b = 0;
    while (b < 64 && (uint64_t(1) << b) < d) b++;
    return b;
}

alto_status make_plan(int nmodes, const uint64_t *dims, alto_info_t *info, LinePlan *lp) {
    if (nmodes < 1 || nmodes > ALTO_MAX_MODES)
        return fail(ALTO_ERR_ARG, "nmodes must be in 1.." + std::to_string(ALTO_MAX_MODES));
    if (!dims) return fail(ALTO_ERR_ARG, "dims is NULL");
    alto_info_t in;
    memset(&in, 0, sizeof(in));
    in.nmodes = nmodes;
    int total = 0, maxb = 0;
    for (int n = 0; n < nmodes; n++) {
        if (dims[n] == 0 || dims[n] > (uint64_t(1) << 31))
            return fail(ALTO_ERR_ARG, "dims[" + std::to_string(n) + "] must be in 1..2^31");
        in.dims[n] = dims[n];
        in.nbits[n] = ceil_log2(dims[n]);
        total += in.nbits[n];
        maxb = std::max(maxb, in.nbits[n]);
    }
    if (total > 128) return fail(ALTO_ERR_INDEX_BITS, "ALTO index needs " + std::to_string(total) + " > 128 bits");
    int order[ALTO_MAX_MODES];
    for (int n = 0; n < nmodes; n++) order[n] = n;
    std::stable_sort(order, order + nmodes, [&](int a, int b) { return dims[a] < dims[b]; });
    int p = 0;
    for (int l = 0; l < maxb; l++) {
        for (int k = 0; k < nmodes; k++) {
            const int n = order[k];
            if (in.nbits[n] > l) {
                if (p < 64) in.mask_lo[n] |= uint64_t(1) << p;
                else in.mask_hi[n] |= uint64_t(1) << (p - 64);
                p++;
            }
        }
    }
    in.index_bits = total;
    in.index_words = total > 64 ? 2 : 1;
    if (lp) {
        memset(lp, 0, sizeof(*lp));
        lp->nmodes = nmodes;
        lp->words = in.index_words;
        for (int n = 0; n < nmodes; n++) {
            ModeMasks &mm = lp->mode[n];
            mm.w[0].mask = in.mask_lo[n];
            mm.w[1].mask = in.mask_hi[n];
            move_masks(in.mask_lo[n], mm.w[0].mv);
            move_masks(in.mask_hi[n], mm.w[1].mv);
            mm.lo_bits = __builtin_popcountll(in.mask_lo[n]);
        }
    }
    if (info) *info = in;
    return ALTO_OK;
}

}  // namespace alto

extern "C" {

alto_status alto_plan_dims(int nmodes, const uint64_t *dims, alto_info_t *out) {
    if (!out) return alto::fail(ALTO_ERR_ARG, "out is NULL");
    return alto::make_plan(nmodes, dims, out, nullptr);
}

alto_status alto_plan_decode_host(const alto_info_t *plan, uint64_t count, const uint64_t *keys, int64_t *coords) {
    if (!plan || (!keys && count) || (!coords && count)) return alto::fail(ALTO_ERR_ARG, "NULL argument");
    alto::LinePlan lp;
    alto_info_t info;
    alto_status st = alto::make_plan(plan->nmodes, plan->dims, &info, &lp);
    if (st != ALTO_OK) return st;
    for (uint64_t i = 0; i < count; i++) {
        const uint64_t lo = keys[2 * i], hi = keys[2 * i + 1];
        for (int n = 0; n < lp.nmodes; n++) {
            const uint32_t c = lp.words == 2 ? alto::extract_mode<2>(lp.mode[n], lo, hi)
                                             : alto::extract_mode<1>(lp.mode[n], lo, hi);
            coords[(uint64_t)n * count + i] = (int64_t)c;
        }
    }
    return ALTO_OK;
}

const char *alto_last_error(void) { return alto::g_last_error.c_str(); }

const char *alto_version(void) { return "alto-mi355x 1.0 gfx950"; }

}  // extern "C"
