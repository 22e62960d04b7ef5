/*
 * Parallel CPU baseline of MTTKRP -- the comparison leg of the benchmark,
 * not part of the checked oracle (which stays single-threaded) and not part
 * of the GPU library.
 *
 * The paper's best COO configuration on CPUs (its experimental setup): the
 * loop over the COO nonzeros split among OpenMP threads, each thread adding
 * into a private copy of the output, the copies summed at the end.  FP64,
 * the same per-nonzero arithmetic as oracle_mttkrp in alto_oracle.c.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int par_threads(void) { return omp_get_max_threads(); }

/* out (dims[mode] x rank, overwritten) = MTTKRP of mode `mode`; returns the
 * number of threads used, or -1 on an argument or allocation error. */
int par_mttkrp(int nmodes, const uint64_t *dims, int64_t nnz, const int64_t *coords, const double *vals, int rank,
               const double *const *factors, int mode, double *out) {
    if (mode < 0 || mode >= nmodes || rank < 1) return -1;
    const int T = omp_get_max_threads();
    const size_t n_out = (size_t)dims[mode] * (size_t)rank;
    double *priv = (double *)calloc((size_t)T * n_out, sizeof(double));
    if (!priv) return -1;
    int used = 1;
#pragma omp parallel
    {
        const int t = omp_get_thread_num();
#pragma omp single
        used = omp_get_num_threads();
        double *o_t = priv + (size_t)t * n_out;
        double *tmp = (double *)malloc(sizeof(double) * (size_t)rank);
#pragma omp for schedule(static)
        for (int64_t x = 0; x < nnz; x++) {
            for (int r = 0; r < rank; r++) tmp[r] = vals[x];
            for (int m = 0; m < nmodes; m++) {
                if (m == mode) continue;
                const double *row = factors[m] + (size_t)coords[(int64_t)m * nnz + x] * (size_t)rank;
                for (int r = 0; r < rank; r++) tmp[r] *= row[r];
            }
            double *o = o_t + (size_t)coords[(int64_t)mode * nnz + x] * (size_t)rank;
            for (int r = 0; r < rank; r++) o[r] += tmp[r];
        }
        free(tmp);
        /* sum the private copies, rows split among the threads */
#pragma omp for schedule(static)
        for (size_t i = 0; i < n_out; i++) {
            double s = 0.0;
            for (int k = 0; k < used; k++) s += priv[(size_t)k * n_out + i];
            out[i] = s;
        }
    }
    free(priv);
    return used;
}
