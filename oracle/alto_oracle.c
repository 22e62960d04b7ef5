/*
 * FP64 CPU oracle for ALTO MTTKRP -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded C written from the paper
 * (Laukemann et al., "Accelerating Sparse Tensor Decomposition Using
 * Adaptive Linearized Representation", arXiv 2403.06348).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the GPU library never does, and this file shares no code with it.
 *
 * Contents
 *   oracle_plan       bit positions of every mode in the ALTO index
 *                     (Sec. "ALTO Tensor Generation", Eq. 1)
 *   oracle_encode     coordinates -> ALTO index, one bit at a time
 *                     (bit-level gather, Fig. "alto_linear"(a))
 *   oracle_decode     ALTO index -> coordinates, one bit at a time
 *                     (bit-level scatter, Fig. "alto_linear"(b))
 *   oracle_order      stable ordering of nonzeros by ALTO index
 *                     (the "ordering" stage of format generation)
 *   oracle_partition  nnz-balanced line segments and their mode intervals
 *                     (Sec. "Workload Partitioning and Scheduling")
 *   oracle_mttkrp     M = X_(n) (A^(1) .. KRP .. A^(N), A^(n) left out)
 *                     as a plain loop over the COO nonzeros
 *                     (Sec. "CP-ALS", sequential MTTKRP algorithm)
 *
 * Readings of the paper taken here (where it is silent or ambiguous):
 *   - coordinates are 0-based (as in the paper's worked example);
 *   - mode n gets ceil(log2 I_n) index bits, 0 bits when I_n = 1;
 *   - within each bit group the modes are ordered by increasing length,
 *     ties broken by mode number, and the shortest mode takes the lowest
 *     bit of the group;  groups are filled from the least significant bit;
 *   - the index is held as two 64-bit words (lo, hi), up to 128 bits;
 *   - ordering is stable: equal indices keep their input order;
 *   - segment l holds nonzeros floor(l*M/L) .. floor((l+1)*M/L)-1;
 *   - MTTKRP overwrites its output (zero, then accumulate).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_MODES 16

/* ceil(log2(d)) for d >= 1; 0 for d == 1. */
static int bits_for_dim(uint64_t d) {
    int b = 0;
    while (b < 64 && ((uint64_t)1 << b) < d) b++;
    return b;
}

/*
 * Bit layout of the ALTO index.
 *   pos[n*64 + l] = position (0..127) in the index of bit l of mode n's
 *                   coordinate, for l < nbits[n].
 *   masks[2*n], masks[2*n+1] = low and high 64-bit words of mode n's mask.
 * Returns the total number of index bits B (Eq. 1), or -1 when B > 128 or
 * an argument is invalid.
 */
int oracle_plan(int nmodes, const uint64_t *dims, int *nbits, int *pos, uint64_t *masks) {
    if (nmodes < 1 || nmodes > ORACLE_MAX_MODES) return -1;
    int order[ORACLE_MAX_MODES];
    int total = 0, maxb = 0;
    for (int n = 0; n < nmodes; n++) {
        if (dims[n] == 0) return -1;
        nbits[n] = bits_for_dim(dims[n]);
        total += nbits[n];
        if (nbits[n] > maxb) maxb = nbits[n];
        order[n] = n;
    }
    if (total > 128) return -1;
    /* modes by increasing length, ties by mode number (insertion sort) */
    for (int i = 1; i < nmodes; i++) {
        int m = order[i], j = i - 1;
        while (j >= 0 && (dims[order[j]] > dims[m] || (dims[order[j]] == dims[m] && order[j] > m))) {
            order[j + 1] = order[j];
            j--;
        }
        order[j + 1] = m;
    }
    for (int n = 0; n < nmodes; n++) {
        masks[2 * n] = 0;
        masks[2 * n + 1] = 0;
        for (int l = 0; l < 64; l++) pos[n * 64 + l] = -1;
    }
    int p = 0;
    for (int l = 0; l < maxb; l++) {          /* bit group l */
        for (int k = 0; k < nmodes; k++) {    /* shortest mode first */
            int n = order[k];
            if (nbits[n] > l) {
                pos[n * 64 + l] = p;
                masks[2 * n + (p >> 6)] |= (uint64_t)1 << (p & 63);
                p++;
            }
        }
    }
    return total;
}

/* keys[2*x] = low word, keys[2*x+1] = high word of nonzero x's index.
 * coords is N x M row-major (coords[n*M + x]).  Returns 0, or the 1-based
 * number of the first nonzero with a coordinate outside its mode. */
int64_t oracle_encode(int nmodes, const uint64_t *dims, int64_t nnz, const int64_t *coords, uint64_t *keys) {
    int nbits[ORACLE_MAX_MODES];
    int pos[ORACLE_MAX_MODES * 64];
    uint64_t masks[2 * ORACLE_MAX_MODES];
    if (oracle_plan(nmodes, dims, nbits, pos, masks) < 0) return -1;
    for (int64_t x = 0; x < nnz; x++) {
        uint64_t lo = 0, hi = 0;
        for (int n = 0; n < nmodes; n++) {
            int64_t c = coords[(int64_t)n * nnz + x];
            if (c < 0 || (uint64_t)c >= dims[n]) return x + 1;
            for (int l = 0; l < nbits[n]; l++) {
                uint64_t bit = ((uint64_t)c >> l) & 1u;
                int p = pos[n * 64 + l];
                if (p < 64) lo |= bit << p;
                else hi |= bit << (p - 64);
            }
        }
        keys[2 * x] = lo;
        keys[2 * x + 1] = hi;
    }
    return 0;
}

int oracle_decode(int nmodes, const uint64_t *dims, int64_t nnz, const uint64_t *keys, int64_t *coords) {
    int nbits[ORACLE_MAX_MODES];
    int pos[ORACLE_MAX_MODES * 64];
    uint64_t masks[2 * ORACLE_MAX_MODES];
    if (oracle_plan(nmodes, dims, nbits, pos, masks) < 0) return -1;
    for (int64_t x = 0; x < nnz; x++) {
        for (int n = 0; n < nmodes; n++) {
            uint64_t c = 0;
            for (int l = 0; l < nbits[n]; l++) {
                int p = pos[n * 64 + l];
                uint64_t w = p < 64 ? keys[2 * x] : keys[2 * x + 1];
                c |= ((w >> (p & 63)) & 1u) << l;
            }
            coords[(int64_t)n * nnz + x] = (int64_t)c;
        }
    }
    return 0;
}

/* ---- ordering: qsort on (key, input position) is a stable sort by key ---- */
struct keyed {
    uint64_t hi, lo;
    int64_t at;
};

static int cmp_keyed(const void *a, const void *b) {
    const struct keyed *u = (const struct keyed *)a, *v = (const struct keyed *)b;
    if (u->hi != v->hi) return u->hi < v->hi ? -1 : 1;
    if (u->lo != v->lo) return u->lo < v->lo ? -1 : 1;
    if (u->at != v->at) return u->at < v->at ? -1 : 1;
    return 0;
}

/* perm[j] = input position of the j-th nonzero in ALTO order. */
int oracle_order(int64_t nnz, const uint64_t *keys, int64_t *perm) {
    struct keyed *t = (struct keyed *)malloc(sizeof(struct keyed) * (size_t)(nnz > 0 ? nnz : 1));
    if (!t) return -1;
    for (int64_t x = 0; x < nnz; x++) {
        t[x].lo = keys[2 * x];
        t[x].hi = keys[2 * x + 1];
        t[x].at = x;
    }
    qsort(t, (size_t)nnz, sizeof(struct keyed), cmp_keyed);
    for (int64_t j = 0; j < nnz; j++) perm[j] = t[j].at;
    free(t);
    return 0;
}

/*
 * Partition the ordered line into L segments of balanced nonzero counts.
 *   starts[l] = floor(l*M/L) for l = 0..L.
 *   intervals[(l*N + n)*2 + 0 / 1] = smallest / largest mode-n coordinate in
 *   segment l (both decoded from the sorted keys).  An empty segment gets
 *   start = UINT64_MAX, end = 0.
 */
int oracle_partition(int nmodes, const uint64_t *dims, int64_t nnz, const uint64_t *sorted_keys, int64_t nseg,
                     int64_t *starts, uint64_t *intervals) {
    if (nseg < 1) return -1;
    for (int64_t l = 0; l <= nseg; l++) {
        /* floor(l*M/L) without overflow for the sizes used here */
        starts[l] = (int64_t)(((__int128)l * nnz) / nseg);
    }
    for (int64_t l = 0; l < nseg; l++) {
        for (int n = 0; n < nmodes; n++) {
            intervals[(l * nmodes + n) * 2 + 0] = UINT64_MAX;
            intervals[(l * nmodes + n) * 2 + 1] = 0;
        }
        for (int64_t x = starts[l]; x < starts[l + 1]; x++) {
            /* decode nonzero x one nonzero at a time */
            int64_t tmp[ORACLE_MAX_MODES];
            oracle_decode(nmodes, dims, 1, sorted_keys + 2 * x, tmp);
            for (int n = 0; n < nmodes; n++) {
                uint64_t v = (uint64_t)tmp[n];
                if (v < intervals[(l * nmodes + n) * 2 + 0]) intervals[(l * nmodes + n) * 2 + 0] = v;
                if (v > intervals[(l * nmodes + n) * 2 + 1]) intervals[(l * nmodes + n) * 2 + 1] = v;
            }
        }
    }
    return 0;
}

/*
 * MTTKRP for mode `mode` over COO nonzeros:
 *   out[i, r] = sum over nonzeros x with i_mode(x) = i of
 *               vals[x] * prod over m != mode (ascending m) of A^(m)[i_m(x), r].
 * factors[m] is row-major dims[m] x rank; factors[mode] is not read.
 * out is dims[mode] x rank, overwritten.
 */
int oracle_mttkrp(int nmodes, const uint64_t *dims, int64_t nnz, const int64_t *coords, const double *vals, int rank,
                  const double *const *factors, int mode, double *out) {
    if (mode < 0 || mode >= nmodes || rank < 1) return -1;
    double *t = (double *)malloc(sizeof(double) * (size_t)rank);
    if (!t) return -1;
    memset(out, 0, sizeof(double) * (size_t)dims[mode] * (size_t)rank);
    for (int64_t x = 0; x < nnz; x++) {
        for (int r = 0; r < rank; r++) t[r] = vals[x];
        for (int m = 0; m < nmodes; m++) {
            if (m == mode) continue;
            const double *row = factors[m] + (size_t)coords[(int64_t)m * nnz + x] * (size_t)rank;
            for (int r = 0; r < rank; r++) t[r] *= row[r];
        }
        double *o = out + (size_t)coords[(int64_t)mode * nnz + x] * (size_t)rank;
        for (int r = 0; r < rank; r++) o[r] += t[r];
    }
    free(t);
    return 0;
}

/*
 * Output rows of MTTKRP for a sample of rows only: for each requested row
 * rows[k] of mode `mode`, out[k, :] is the same sum as in oracle_mttkrp.
 * Scans all nonzeros once; used to check full-size results row by row.
 * rows[] must be sorted ascending and distinct.
 */
int oracle_mttkrp_rows(int nmodes, const uint64_t *dims, int64_t nnz, const int64_t *coords, const double *vals,
                       int rank, const double *const *factors, int mode, int64_t nrows, const int64_t *rows,
                       double *out) {
    (void)dims;
    if (mode < 0 || mode >= nmodes || rank < 1) return -1;
    double *t = (double *)malloc(sizeof(double) * (size_t)rank);
    if (!t) return -1;
    memset(out, 0, sizeof(double) * (size_t)nrows * (size_t)rank);
    for (int64_t x = 0; x < nnz; x++) {
        int64_t i = coords[(int64_t)mode * nnz + x];
        /* binary search for i among the requested rows */
        int64_t lo = 0, hi = nrows;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (rows[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        if (lo >= nrows || rows[lo] != i) continue;
        for (int r = 0; r < rank; r++) t[r] = vals[x];
        for (int m = 0; m < nmodes; m++) {
            if (m == mode) continue;
            const double *row = factors[m] + (size_t)coords[(int64_t)m * nnz + x] * (size_t)rank;
            for (int r = 0; r < rank; r++) t[r] *= row[r];
        }
        double *o = out + (size_t)lo * (size_t)rank;
        for (int r = 0; r < rank; r++) o[r] += t[r];
    }
    free(t);
    return 0;
}

/*
 * CP-APR model update Phi for mode `mode` (Algorithm "alg:cp-apr-mu", the
 * Phi line; Algorithm "fig:subproblem_algo" for the per-nonzero form):
 *   for every nonzero x with coordinates i and value v:
 *     krp[r] = prod over m != mode (ascending m) of A^(m)[i_m, r]
 *     d      = sum_r B[i_mode, r] * krp[r]         (the model at x)
 *     out[i_mode, r] += v / max(d, eps) * krp[r]
 * factors[m] and B (dims[mode] x rank) are row-major; out is overwritten.
 */
int oracle_phi(int nmodes, const uint64_t *dims, int64_t nnz, const int64_t *coords, const double *vals, int rank,
               const double *const *factors, const double *B, int mode, double eps, double *out) {
    if (mode < 0 || mode >= nmodes || rank < 1) return -1;
    double *krp = (double *)malloc(sizeof(double) * (size_t)rank);
    if (!krp) return -1;
    memset(out, 0, sizeof(double) * (size_t)dims[mode] * (size_t)rank);
    for (int64_t x = 0; x < nnz; x++) {
        for (int r = 0; r < rank; r++) krp[r] = 1.0;
        for (int m = 0; m < nmodes; m++) {
            if (m == mode) continue;
            const double *row = factors[m] + (size_t)coords[(int64_t)m * nnz + x] * (size_t)rank;
            for (int r = 0; r < rank; r++) krp[r] *= row[r];
        }
        const int64_t i = coords[(int64_t)mode * nnz + x];
        const double *b = B + (size_t)i * (size_t)rank;
        double d = 0.0;
        for (int r = 0; r < rank; r++) d += b[r] * krp[r];
        const double s = vals[x] / (d > eps ? d : eps);
        double *o = out + (size_t)i * (size_t)rank;
        for (int r = 0; r < rank; r++) o[r] += s * krp[r];
    }
    free(krp);
    return 0;
}

/*
 * Rows of Pi for mode `mode`, one per nonzero in input order (the Pi line of
 * Algorithm "alg:cp-apr-mu", computed only for the nonzeros):
 *   pi[x, r] = prod over m != mode (ascending m) of A^(m)[i_m(x), r].
 */
int oracle_pi(int nmodes, int64_t nnz, const int64_t *coords, int rank, const double *const *factors, int mode,
              double *pi) {
    if (mode < 0 || mode >= nmodes || rank < 1) return -1;
    for (int64_t x = 0; x < nnz; x++) {
        double *p = pi + (size_t)x * (size_t)rank;
        for (int r = 0; r < rank; r++) p[r] = 1.0;
        for (int m = 0; m < nmodes; m++) {
            if (m == mode) continue;
            const double *row = factors[m] + (size_t)coords[(int64_t)m * nnz + x] * (size_t)rank;
            for (int r = 0; r < rank; r++) p[r] *= row[r];
        }
    }
    return 0;
}
