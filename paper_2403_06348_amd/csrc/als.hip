// One CP-ALS sweep on the GPU (Algorithm "alg:cp-als" of the paper).
//
// Per mode n:  V = Hadamard product of the Grams of the other factors;
// M = MTTKRP(n); A^(n) = M V^-1; lambda = column 2-norms of A^(n); columns
// divided by lambda.  The R x R work (Grams, Cholesky, inverse, lambda) is
// FP64; the I x R matrices are FP32 (FP64 arithmetic, FP32 storage).
//
// Kernels
//   k_gram_rows      partial Grams A^T A of row chunks (FP64 accumulation)
//   k_gram_reduce    sum of the partials (fixed order, deterministic)
//   k_als_prepare    one workgroup: V, Cholesky V = L L^T, W = L^-T L^-1;
//                    if a pivot is at rounding level, W = pseudo-inverse from
//                    a cyclic Jacobi eigendecomposition (flag bit n set)
//   k_gram_rows<.., true>  A^(n) = M W row by row, plus partial Grams of A^(n)
//   k_als_finalize   lambda_r = sqrt(G_rr), Gram of the normalized factor
//   k_als_normalize  A^(n)(:, r) /= lambda_r, BF16 shadow refresh
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "alto_internal.h"
#include "device_util.h"
#include "memory.h"
#include "mttkrp.h"

namespace alto {
namespace {

constexpr int kThreads = 256;
constexpr int kPartials = kSweepPartials;  // partial Gram blocks
constexpr int kMaxSweepRank = 64;
constexpr int kMaxPairs = kMaxSweepRank / 2;  // Jacobi rotations per step
static_assert(kThreads == 8 * kMaxPairs && kMaxSweepRank <= 64, "Jacobi step thread layout: 32 x 8 blocks, 4 x 64 Q rows");
__device__ inline uint16_t f32_to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));  // inf / nan
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

// Partial Grams over row chunks, register-tiled.  A block stages 256
// consecutive rows (FP32, one per thread) in LDS; for APPLY it first forms
// each row of A = M W (thread per row, FP64 accumulation, W read from LDS
// as broadcasts), stores it as FP32 to A and back into LDS.  Then every
// thread accumulates one 4 x 4 tile of sum_i a_i a_i^T over its share of
// the chunk's rows in FP64.  At the end the row groups' tiles are added in
// a fixed order and the block writes its partial R x R Gram.
// RB: rank bucket (8, 16, 32, 64), R <= RB, R a multiple of 4.
// blk / nblk: this workgroup's chunk of the rows and the chunk count (the
// partial Gram it writes).  shadow (not APPLY): also store the BF16 copy of
// the staged rows.
template <int RB, bool APPLY>
__device__ inline void gram_rows_body(const float *__restrict__ src, const double *__restrict__ W,
                                      float *__restrict__ A, uint64_t I, int R, double *__restrict__ partials,
                                      uint16_t *__restrict__ shadow, unsigned blk, unsigned nblk) {
    constexpr int STR = RB + 4;             // LDS row stride (floats), 16-byte aligned
    constexpr int TPR = RB / 4;             // 4 x 4 tiles per Gram row
    constexpr int TB = TPR * TPR;           // tiles of the Gram
    constexpr int G = kThreads / TB;        // row groups
    constexpr int SA = kThreads * STR > 8192 ? kThreads * STR : 8192;  // floats; >= 32 KiB for the tile sums
    __shared__ __align__(16) float sa[SA];
    __shared__ __align__(16) double sw[APPLY ? RB * RB : 1];
    const int tid = threadIdx.x;
    const int t = tid % TB, g = tid / TB;
    const int tr = t / TPR, ts = t % TPR;
    const bool tile_ok = 4 * tr < R && 4 * ts < R;
    if (APPLY)
        for (int e = tid; e < R * R; e += kThreads) sw[(e / R) * RB + e % R] = W[e];
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int y = 0; y < 4; y++) acc[x][y] = 0.0;
    const uint64_t per = (I + nblk - 1) / nblk;
    const uint64_t a = (uint64_t)blk * per;
    const uint64_t b = a + per < I ? a + per : I;
    const int q4 = R / 4;
    for (uint64_t c = a; c < b; c += kThreads) {
        const int rows = (int)((b - c) < (uint64_t)kThreads ? (b - c) : (uint64_t)kThreads);
        __syncthreads();
        const float4 *s4 = (const float4 *)(src + c * R);
        for (int v = tid; v < rows * q4; v += kThreads) {
            const int row = v / q4, q = v - row * q4;
            const float4 f = s4[v];
            *(float4 *)(sa + row * STR + 4 * q) = f;
            if (!APPLY && shadow) {
                const uint32_t lo = (uint32_t)f32_to_bf16_rne(f.x) | ((uint32_t)f32_to_bf16_rne(f.y) << 16);
                const uint32_t hi = (uint32_t)f32_to_bf16_rne(f.z) | ((uint32_t)f32_to_bf16_rne(f.w) << 16);
                ((uint2 *)(shadow + c * R))[v] = make_uint2(lo, hi);
            }
        }
        __syncthreads();
        if (APPLY && RB >= 32) {
            // register tiles of A = M W: thread (rg, cg) computes rows
            // 4 rg .. 4 rg + 3 and columns cg*CG .. +CG-1, so each W value
            // read from LDS serves four rows
            constexpr int CG = RB / 4;
            const int cg = tid & 3, rg = tid >> 2;
            double o[4][CG];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < CG; j++) o[i][j] = 0.0;
            if (4 * rg < rows) {
                for (int k0 = 0; k0 < R; k0 += 4) {
                    float4 m4[4];
#pragma unroll
                    for (int i = 0; i < 4; i++) m4[i] = *(const float4 *)(sa + (4 * rg + i) * STR + k0);
#pragma unroll
                    for (int kk = 0; kk < 4; kk++) {
                        const double *wk = sw + (k0 + kk) * RB + cg * CG;
                        double mk[4];
#pragma unroll
                        for (int i = 0; i < 4; i++)
                            mk[i] = (double)(kk == 0 ? m4[i].x : kk == 1 ? m4[i].y : kk == 2 ? m4[i].z : m4[i].w);
#pragma unroll
                        for (int j = 0; j < CG; j += 2) {
                            const double2 w2 = *(const double2 *)(wk + j);
#pragma unroll
                            for (int i = 0; i < 4; i++) {
                                o[i][j] = fma(mk[i], w2.x, o[i][j]);
                                o[i][j + 1] = fma(mk[i], w2.y, o[i][j + 1]);
                            }
                        }
                    }
                }
            }
            __syncthreads();  // every tile has read its rows of M from sa
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int row = 4 * rg + i;
                if (row >= rows) break;
                float4 *dst = (float4 *)(A + (c + row) * R);
#pragma unroll
                for (int j = 0; j < CG; j += 4) {
                    const int col = cg * CG + j;
                    if (col < R) {
                        const float4 f = make_float4((float)o[i][j], (float)o[i][j + 1], (float)o[i][j + 2],
                                                     (float)o[i][j + 3]);
                        dst[col / 4] = f;
                        *(float4 *)(sa + row * STR + col) = f;
                    }
                }
            }
        } else if (APPLY && tid < rows) {
            float m[RB];
#pragma unroll
            for (int k = 0; k < RB; k += 4) {
                const float4 v = k < R ? *(const float4 *)(sa + tid * STR + k) : make_float4(0.f, 0.f, 0.f, 0.f);
                m[k] = v.x;
                m[k + 1] = v.y;
                m[k + 2] = v.z;
                m[k + 3] = v.w;
            }
            // output columns in blocks of at most 32 (FP64 accumulators),
            // the rank loop unrolled over the bucket so that m stays in
            // registers
            constexpr int CB = RB < 32 ? RB : 32;
            float4 *dst = (float4 *)(A + (c + tid) * R);
#pragma unroll
            for (int j0 = 0; j0 < RB; j0 += CB) {
                if (j0 < R) {
                    double o[CB];
#pragma unroll
                    for (int j = 0; j < CB; j++) o[j] = 0.0;
#pragma unroll
                    for (int k = 0; k < RB; k++) {
                        if (k < R) {
                            const double mk = (double)m[k];
                            const double *wk = sw + k * RB + j0;
#pragma unroll
                            for (int j = 0; j < CB; j += 2) {
                                if (j0 + j < R) {
                                    const double2 w2 = *(const double2 *)(wk + j);
                                    o[j] = fma(mk, w2.x, o[j]);
                                    o[j + 1] = fma(mk, w2.y, o[j + 1]);
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int j = 0; j < CB; j += 4) {
                        if (j0 + j < R) {
                            const float4 f = make_float4((float)o[j], (float)o[j + 1], (float)o[j + 2], (float)o[j + 3]);
                            dst[(j0 + j) / 4] = f;
                            *(float4 *)(sa + tid * STR + j0 + j) = f;
                        }
                    }
                }
            }
        }
        if (APPLY) __syncthreads();
        if (tile_ok) {
            for (int i = g; i < rows; i += G) {
                const float4 x = *(const float4 *)(sa + i * STR + 4 * tr);
                const float4 y = *(const float4 *)(sa + i * STR + 4 * ts);
                const double xv[4] = {x.x, x.y, x.z, x.w}, yv[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
                for (int u = 0; u < 4; u++)
#pragma unroll
                    for (int w = 0; w < 4; w++) acc[u][w] = fma(xv[u], yv[w], acc[u][w]);
            }
        }
    }
    __syncthreads();
    // tile sums of the row groups, then their fixed-order total per entry
    double *red = (double *)sa;  // G x TB x 16 doubles = 32 KiB
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
        for (int w = 0; w < 4; w++) red[((size_t)g * TB + t) * 16 + u * 4 + w] = acc[u][w];
    __syncthreads();
    double *o = partials + (uint64_t)blk * R * R;
    for (int e = tid; e < R * R; e += kThreads) {
        const int r = e / R, c2 = e % R;
        const int tt = (r / 4) * TPR + c2 / 4, pos = (r % 4) * 4 + c2 % 4;
        double sum = 0.0;
        for (int k = 0; k < G; k++) sum += red[((size_t)k * TB + tt) * 16 + pos];
        o[e] = sum;
    }
}

template <int RB, bool APPLY>
__global__ __launch_bounds__(kThreads) void k_gram_rows(const float *__restrict__ src, const double *__restrict__ W,
                                                        float *__restrict__ A, uint64_t I, int R,
                                                        double *__restrict__ partials) {
    gram_rows_body<RB, APPLY>(src, W, A, I, R, partials, nullptr, blockIdx.x, gridDim.x);
}

// G = sum of the np partial R x R blocks.  Block b owns entries
// [64 b, 64 b + 64); its 4 waves take every 4th partial with two independent
// sums each, then add their results in a fixed order (deterministic).
__device__ inline void gram_reduce_block(const double *__restrict__ partials, int np, int R, double *__restrict__ G,
                                         int eb) {
    __shared__ double red[4][64];
    const int rr = R * R;
    const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int e = eb * 64 + t;
    double s0 = 0.0, s1 = 0.0;
    if (e < rr) {
        int p = w;
        for (; p + 4 < np; p += 8) {
            s0 += partials[(uint64_t)p * rr + e];
            s1 += partials[(uint64_t)(p + 4) * rr + e];
        }
        for (; p < np; p += 4) s0 += partials[(uint64_t)p * rr + e];
    }
    red[w][t] = s0 + s1;
    __syncthreads();
    if (w == 0 && e < rr) G[e] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

__global__ __launch_bounds__(kThreads) void k_gram_reduce(const double *__restrict__ partials, int np, int R,
                                                          double *__restrict__ G) {
    gram_reduce_block(partials, np, R, G, blockIdx.x);
}

inline unsigned gram_reduce_blocks(int R) { return (unsigned)((R * R + 63) / 64); }

// One workgroup.  grams: N x R x R; W: R x R output; flags bit n on
// fallback; sm: 3 R x R doubles of LDS.
// LDS of the solve preparation: three R x R FP64 matrices, row stride R + 1.
inline size_t prepare_lds_bytes(int R) { return (size_t)3 * R * (R + 1) * sizeof(double); }

// Rt <= R: the model's true rank.  Columns Rt..R-1 are zero padding (ranks
// are stored as multiples of 4); their Gram rows and columns are zero, so V
// gets an identity block scaled to its largest diagonal entry there: the
// solve then leaves the padding columns of A = M V^-1 at zero (M is zero
// there too) and the true block is solved exactly as without padding.
__device__ inline void als_prepare(const double *__restrict__ grams, int N, int n, int R, int Rt,
                                   double *__restrict__ W, uint32_t *flags, double *sm) {
    // R x R matrices in LDS with row stride R + 1: walks down a column then
    // touch every bank instead of one
    const int LD = R + 1;
    double *V = sm;           // R x R
    double *L = sm + R * LD;  // R x R (Cholesky factor, then inverse / eigenvectors)
    double *T = L + R * LD;   // R x R scratch
    __shared__ int not_spd;
    __shared__ double vmax;
    const int tid = threadIdx.x;
    for (int e = tid; e < R * R; e += kThreads) {
        double v = 1.0;
        if (e / R < Rt && e % R < Rt) {
            for (int m = 0; m < N; m++)
                if (m != n) v *= grams[(uint64_t)m * R * R + e];
        } else {
            v = 0.0;
        }
        V[(e / R) * LD + e % R] = v;
        L[(e / R) * LD + e % R] = 0.0;
    }
    if (tid == 0) not_spd = 0;
    __syncthreads();
    if (tid == 0) {
        double mx = 0.0;
        for (int k = 0; k < Rt; k++) mx = fmax(mx, V[k * LD + k]);
        vmax = mx;
        for (int k = Rt; k < R; k++) V[k * LD + k] = mx > 0.0 ? mx : 1.0;
    }
    __syncthreads();
    const double tol = (double)R * 2.220446049250313e-16 * vmax;
    // left-looking Cholesky, one column at a time, rows in parallel
    for (int k = 0; k < R; k++) {
        for (int i = k + tid; i < R; i += kThreads) {
            double t = V[i * LD + k];
#pragma unroll 4
            for (int j = 0; j < k; j++) t -= L[i * LD + j] * L[k * LD + j];
            T[i] = t;
        }
        __syncthreads();
        const double d = T[k];
        if (!(d > tol)) {
            if (tid == 0) not_spd = 1;
            __syncthreads();
            break;
        }
        const double lk = sqrt(d);
        for (int i = k + tid; i < R; i += kThreads) L[i * LD + k] = (i == k) ? lk : T[i] / lk;
        __syncthreads();
    }
    __syncthreads();
    if (!not_spd) {
        // columns of L^-1 by forward substitution (column j per thread)
        double *Li = T;  // reuse as R x R
        for (int j = tid; j < R; j += kThreads) {
            for (int i = 0; i < R; i++) {
                double s = (i == j) ? 1.0 : 0.0;
#pragma unroll 4
                for (int k = j; k < i; k++) s -= L[i * LD + k] * Li[k * LD + j];
                Li[i * LD + j] = (i < j) ? 0.0 : s / L[i * LD + i];
            }
        }
        __syncthreads();
        // W = L^-T L^-1
        for (int e = tid; e < R * R; e += kThreads) {
            const int r = e / R, s = e % R;
            double w = 0.0;
#pragma unroll 4
            for (int k = (r > s ? r : s); k < R; k++) w += Li[k * LD + r] * Li[k * LD + s];
            W[e] = w;
        }
        return;
    }
    // ---- fallback: symmetric eigendecomposition by parallel cyclic Jacobi.
    // A step rotates R/2 disjoint index pairs at once (round-robin pairing:
    // over R-1 steps every pair meets once, a full sweep).  Rotations on
    // disjoint pairs commute, and each pair's own 2x2 block is touched by its
    // rotation only, so a step equals applying its rotations one after
    // another.  R is even (ranks are multiples of 4), so every index is in
    // exactly one pair and A <- J^T A J splits into independent 2x2 blocks
    // (pair of the rows, pair of the columns): each block is rotated by its
    // column pair, then by its row pair, in one pass.
    double *Aj = T;  // working copy
    double *Q = L;
    for (int e = tid; e < R * LD; e += kThreads) {
        Aj[e] = V[e];
        Q[e] = (e / LD == e % LD) ? 1.0 : 0.0;
    }
    __shared__ double rot[kMaxPairs][2];
    __shared__ int pair[kMaxPairs][2];
    __shared__ int rotated;
    __shared__ double fro_part[kThreads / 64];
    const int np = R / 2;
    // threshold Jacobi: a pair is rotated only while its off-diagonal entry
    // exceeds the FP64 rounding level of V (eps * ||V||_F, the backward error
    // of a stable eigensolver); a sweep that rotates nothing ends the
    // iteration.  A relative stopping rule on the off-diagonal mass stalls at
    // that noise level (rotations among the negligible eigenvalues keep
    // regenerating it), while the pseudo-inverse drops those eigenvalues.
    {
        double f2 = 0.0;
        for (int e = tid; e < R * R; e += kThreads) f2 += V[(e / R) * LD + e % R] * V[(e / R) * LD + e % R];
#pragma unroll
        for (int w = 32; w > 0; w >>= 1) f2 += __shfl_xor(f2, w, 64);
        if ((tid & 63) == 0) fro_part[tid >> 6] = f2;
    }
    __syncthreads();
    double fro2 = 0.0;
    for (int w = 0; w < kThreads / 64; w++) fro2 += fro_part[w];
    const double rot_tol = 2.220446049250313e-16 * sqrt(fro2);
    for (int sweep = 0; sweep < 40; sweep++) {
        __syncthreads();  // every thread has read the previous sweep's flag
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int step = 0; step < R - 1; step++) {
            if (tid < np) {
                // round-robin pairing: index R-1 stays, the others rotate;
                // step + tid < 3R/2 and step - tid + R - 1 < 2R, so one
                // subtraction reduces each modulo R - 1
                int p = step + tid, q = step - tid + (R - 1);
                if (p >= R - 1) p -= R - 1;
                if (q >= R - 1) q -= R - 1;
                if (tid == 0) {
                    p = R - 1;
                    q = step;
                }
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, sn = 0.0;
                const double apq = Aj[p * LD + q];
                if (fabs(apq) > rot_tol) {
                    const double theta = (Aj[q * LD + q] - Aj[p * LD + p]) / (2.0 * apq);
                    const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                    c = 1.0 / sqrt(t * t + 1.0);
                    sn = t * c;
                    atomicOr(&rotated, 1);
                }
                rot[tid][0] = c;
                rot[tid][1] = sn;
                pair[tid][0] = p;
                pair[tid][1] = q;
            }
            __syncthreads();
            // blocks (row pair a, column pair b): thread (a, b0) of a 32 x 8
            // grid takes column pairs b0, b0 + 8, b0 + 16, b0 + 24 (R <= 64), and
            // Q's rows k = tid mod 64 for pairs w0, w0 + 4, ..., w0 + 28.  Each
            // thread issues all of its loads before its stores; the blocks and
            // Q entries of different threads and pairs are disjoint.
            {
                constexpr int NB = kMaxPairs / 8, NQ = kMaxPairs / 4;
                const int a = tid >> 3, b0 = tid & 7;
                if (a < np) {
                    const double ca = rot[a][0], sa = rot[a][1];
                    const int p = pair[a][0], q = pair[a][1];
                    double blk[NB][4], cb[NB], sb[NB];
                    int u[NB], v[NB];
#pragma unroll
                    for (int j = 0; j < NB; j++) {
                        const int bb = b0 + 8 * j;
                        cb[j] = 1.0;
                        sb[j] = 0.0;
                        u[j] = v[j] = 0;
                        if (bb < np) {
                            cb[j] = rot[bb][0];
                            sb[j] = rot[bb][1];
                            u[j] = pair[bb][0];
                            v[j] = pair[bb][1];
                            blk[j][0] = Aj[p * LD + u[j]];
                            blk[j][1] = Aj[p * LD + v[j]];
                            blk[j][2] = Aj[q * LD + u[j]];
                            blk[j][3] = Aj[q * LD + v[j]];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < NB; j++) {
                        if (b0 + 8 * j >= np || (sa == 0.0 && sb[j] == 0.0)) continue;
                        const double xpu = cb[j] * blk[j][0] - sb[j] * blk[j][1];
                        const double xpv = sb[j] * blk[j][0] + cb[j] * blk[j][1];
                        const double xqu = cb[j] * blk[j][2] - sb[j] * blk[j][3];
                        const double xqv = sb[j] * blk[j][2] + cb[j] * blk[j][3];
                        Aj[p * LD + u[j]] = ca * xpu - sa * xqu;
                        Aj[q * LD + u[j]] = sa * xpu + ca * xqu;
                        Aj[p * LD + v[j]] = ca * xpv - sa * xqv;
                        Aj[q * LD + v[j]] = sa * xpv + ca * xqv;
                    }
                }
                const int w0 = tid >> 6, k = tid & 63;
                if (k < R) {
                    double qp[NQ], qq[NQ];
#pragma unroll
                    for (int j = 0; j < NQ; j++) {
                        const int w = w0 + 4 * j;
                        if (w < np) {
                            qp[j] = Q[k * LD + pair[w][0]];
                            qq[j] = Q[k * LD + pair[w][1]];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < NQ; j++) {
                        const int w = w0 + 4 * j;
                        if (w >= np) continue;
                        const double c = rot[w][0], sn = rot[w][1];
                        if (sn == 0.0) continue;
                        Q[k * LD + pair[w][0]] = c * qp[j] - sn * qq[j];
                        Q[k * LD + pair[w][1]] = sn * qp[j] + c * qq[j];
                    }
                }
            }
            __syncthreads();
        }
        if (rotated == 0) break;  // uniform: read after the step's barrier
    }
    __shared__ double emax;
    if (tid == 0) {
        double mx = 0.0;
        for (int k = 0; k < R; k++) mx = fmax(mx, fabs(Aj[k * LD + k]));
        emax = mx;
        atomicOr(flags, 1u << n);
    }
    __syncthreads();
    const double cut = (double)R * 2.220446049250313e-16 * emax;
    __shared__ double ilam[kMaxSweepRank];  // 1/lambda_k, 0 for dropped eigenvalues
    for (int k = tid; k < R; k += kThreads) {
        const double lam = Aj[k * LD + k];
        ilam[k] = lam > cut ? 1.0 / lam : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < R * R; e += kThreads) {
        const int r = e / R, s = e % R;
        double w = 0.0;
#pragma unroll 4
        for (int k = 0; k < R; k++) w += Q[r * LD + k] * Q[s * LD + k] * ilam[k];
        W[e] = w;
    }
}

__global__ __launch_bounds__(kThreads) void k_als_prepare(const double *__restrict__ grams, int N, int n, int R,
                                                          int Rt, double *__restrict__ W, uint32_t *flags) {
    extern __shared__ double sm[];
    als_prepare(grams, N, n, R, Rt, W, flags, sm);
}

// Gn holds the Gram of the updated (unnormalized) factor: lambda = the
// column norms, then Gn is rescaled in place to the normalized factor's Gram.
__device__ inline void als_finalize(double *__restrict__ Gn, int R, double *__restrict__ lam_ws,
                                    double *__restrict__ lam_out) {
    __shared__ double lam[kMaxSweepRank];
    for (int r = threadIdx.x; r < R; r += kThreads) {
        const double l = sqrt(fmax(Gn[r * R + r], 0.0));
        lam[r] = l;
        lam_ws[r] = l;
        if (lam_out) lam_out[r] = l;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < R * R; e += kThreads) {
        const int r = e / R, s = e % R;
        const double d = lam[r] * lam[s];
        Gn[e] = d > 0.0 ? Gn[e] / d : 0.0;
    }
}

__global__ __launch_bounds__(kThreads) void k_als_finalize(double *__restrict__ Gn, int R, double *__restrict__ lam_ws,
                                                           double *__restrict__ lam_out) {
    als_finalize(Gn, R, lam_ws, lam_out);
}

// A(:, c) /= lambda_c over elements start, start + stride, ...; the column
// advances by stride mod R per step (no division per element).
__device__ inline void als_normalize(float *__restrict__ A, uint64_t I, int R, const double *__restrict__ lam,
                                     uint16_t *__restrict__ shadow, uint64_t start, uint64_t stride) {
    const uint64_t n = I * R;
    if (start >= n) return;
    const uint32_t step = (uint32_t)(stride % (uint64_t)R);
    uint32_t c = (uint32_t)(start % (uint64_t)R);
    for (uint64_t t = start; t < n; t += stride) {
        const double l = lam[c];
        float v = A[t];
        if (l > 0.0) v = (float)((double)v / l);
        A[t] = v;
        if (shadow) shadow[t] = f32_to_bf16_rne(v);
        c += step;
        if (c >= (uint32_t)R) c -= (uint32_t)R;
    }
}

__global__ void k_als_normalize(float *__restrict__ A, uint64_t I, int R, const double *__restrict__ lam,
                                uint16_t *__restrict__ shadow) {
    als_normalize(A, I, R, lam, shadow, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x,
                  (uint64_t)gridDim.x * blockDim.x);
}

// ---- the same R x R steps for many sweeps at once: one launch per step,
// workgroups indexed by job (blockIdx.x) and, where a job has more work
// than one workgroup, by part (blockIdx.y)
struct SweepJob {
    const double *grams;     // N x R x R Grams
    double *W;               // R x R solve operator
    uint32_t *flags;         // pseudo-inverse fallback flags
    double *partials;        // P partial R x R Grams
    double *G;               // Gram the partials are summed into
    double *lam_ws;          // lambda of the mode (workspace)
    double *lam_out;         // caller's lambda (last mode) or null
    float *A;                // factor to normalize
    uint16_t *shadow;        // its BF16 shadow or null
    const float *M;          // the mode's MTTKRP result
    uint64_t I;
    int N, n, R, P;
    uint32_t blk0;           // first workgroup of the job in its Gram launch
};

__global__ __launch_bounds__(kThreads) void k_als_prepare_b(const SweepJob *__restrict__ jobs) {
    extern __shared__ double sm[];
    const SweepJob &j = jobs[blockIdx.x];
    als_prepare(j.grams, j.N, j.n, j.R, j.R, j.W, j.flags, sm);
}

// Row-chunk Grams of many jobs of one rank bucket in one launch: workgroup
// w works on job k where blk0_k <= w < blk0_k + P_k (blk0 ascending).  Not
// APPLY: Gram of the factor A (and its BF16 shadow); APPLY: A = M W and the
// Gram of the new A.
template <int RB, bool APPLY>
__global__ __launch_bounds__(kThreads) void k_gram_rows_b(const SweepJob *__restrict__ jobs, int nj) {
    const unsigned w = blockIdx.x;
    int lo = 0, hi = nj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].blk0 <= w) lo = mid;
        else hi = mid - 1;
    }
    const SweepJob &j = jobs[lo];
    gram_rows_body<RB, APPLY>(APPLY ? j.M : j.A, j.W, j.A, j.I, j.R, j.partials, APPLY ? nullptr : j.shadow,
                              w - j.blk0, (unsigned)j.P);
}

__global__ __launch_bounds__(kThreads) void k_gram_reduce_b(const SweepJob *__restrict__ jobs) {
    const SweepJob &j = jobs[blockIdx.x];
    if ((int)blockIdx.y * 64 >= j.R * j.R) return;  // whole workgroup
    gram_reduce_block(j.partials, j.P, j.R, j.G, blockIdx.y);
}

__global__ __launch_bounds__(kThreads) void k_als_finalize_b(const SweepJob *__restrict__ jobs) {
    const SweepJob &j = jobs[blockIdx.x];
    als_finalize(j.G, j.R, j.lam_ws, j.lam_out);
}

// Every workgroup takes part in every job (grid-stride within each job), so
// a job's share of the grid does not depend on its position or size.
__global__ void k_als_normalize_b(const SweepJob *__restrict__ jobs, int nj) {
    const uint64_t start = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (int k = 0; k < nj; k++) {
        const SweepJob &j = jobs[k];
        als_normalize(j.A, j.I, j.R, j.lam_ws, j.shadow, start, stride);
    }
}

__global__ void k_to_bf16(const float *__restrict__ A, uint64_t n, uint16_t *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) out[t] = f32_to_bf16_rne(A[t]);
}

// Rank bucket of the register-tiled Gram kernels.
int rank_bucket(int R) { return R <= 8 ? 8 : R <= 16 ? 16 : R <= 32 ? 32 : 64; }

template <bool APPLY>
void launch_gram_rows(int R, unsigned P, hipStream_t s, const float *src, const double *W, float *A, uint64_t I,
                      double *partials) {
    switch (rank_bucket(R)) {
        case 8: hipLaunchKernelGGL((k_gram_rows<8, APPLY>), dim3(P), dim3(kThreads), 0, s, src, W, A, I, R, partials); break;
        case 16: hipLaunchKernelGGL((k_gram_rows<16, APPLY>), dim3(P), dim3(kThreads), 0, s, src, W, A, I, R, partials); break;
        case 32: hipLaunchKernelGGL((k_gram_rows<32, APPLY>), dim3(P), dim3(kThreads), 0, s, src, W, A, I, R, partials); break;
        default: hipLaunchKernelGGL((k_gram_rows<64, APPLY>), dim3(P), dim3(kThreads), 0, s, src, W, A, I, R, partials); break;
    }
}

template <bool APPLY>
void launch_gram_rows_b(int rb, unsigned blocks, hipStream_t s, const SweepJob *jobs, int nj) {
    switch (rb) {
        case 8: hipLaunchKernelGGL((k_gram_rows_b<8, APPLY>), dim3(blocks), dim3(kThreads), 0, s, jobs, nj); break;
        case 16: hipLaunchKernelGGL((k_gram_rows_b<16, APPLY>), dim3(blocks), dim3(kThreads), 0, s, jobs, nj); break;
        case 32: hipLaunchKernelGGL((k_gram_rows_b<32, APPLY>), dim3(blocks), dim3(kThreads), 0, s, jobs, nj); break;
        default: hipLaunchKernelGGL((k_gram_rows_b<64, APPLY>), dim3(blocks), dim3(kThreads), 0, s, jobs, nj); break;
    }
}

unsigned partial_blocks(uint64_t I) {
    uint64_t p = (I + 255) / 256;
    if (p > kPartials) p = kPartials;
    if (p < 1) p = 1;
    return (unsigned)p;
}

// Device table of the batched sweep's per-job steps, per (device, stream).
struct SweepStage {
    SweepJob *dev = nullptr;
    size_t cap = 0;
};
std::mutex g_sweep_stage_mu;
std::map<std::pair<int, hipStream_t>, SweepStage> g_sweep_stage;

alto_status upload_sweep_jobs(const std::vector<SweepJob> &host, hipStream_t s, SweepJob **out) {
    int dev = 0;
    ALTO_HIP(hipGetDevice(&dev));
    SweepStage *st;
    {
        std::lock_guard<std::mutex> lk(g_sweep_stage_mu);
        st = &g_sweep_stage[{dev, s}];
    }
    if (st->cap < host.size()) {
        if (st->dev) {
            dev_free_after(st->dev, s);
            st->dev = nullptr;
            st->cap = 0;
        }
        if (dev_alloc((void **)&st->dev, host.size() * sizeof(SweepJob)) != hipSuccess)
            return fail(ALTO_ERR_OOM, "batched sweep staging allocation failed");
        st->cap = host.size();
    }
    ALTO_HIP(hipMemcpyAsync(st->dev, host.data(), host.size() * sizeof(SweepJob), hipMemcpyHostToDevice, s));
    *out = st->dev;
    return ALTO_OK;
}

}  // namespace

// Checks and workspace of one sweep; resets its fallback flags.
alto_status sweep_setup(alto_tensor *h, int rank, int fdt, float *const *factors, const double *lambda,
                        hipStream_t s) {
    ALTO_CHECK_HANDLE(h);
    h->stream = s;
    const int N = h->info.nmodes;
    const int R = rank;
    if (R < 4 || R > kMaxSweepRank || R % 4) return fail(ALTO_ERR_ARG, "sweep rank must be in 1..64");
    if (fdt != ALTO_F32 && fdt != ALTO_BF16) return fail(ALTO_ERR_ARG, "bad factor dtype");
    if (!factors || !lambda) return fail(ALTO_ERR_ARG, "factors/lambda is NULL");
    for (int m = 0; m < N; m++) {
        if (!factors[m]) return fail(ALTO_ERR_ARG, "factors[" + std::to_string(m) + "] is NULL");
        if ((uintptr_t)factors[m] & 15) return fail(ALTO_ERR_ARG, "factors must be 16-byte aligned");
    }
    uint64_t maxI = 0;
    for (int m = 0; m < N; m++) maxI = h->info.dims[m] > maxI ? h->info.dims[m] : maxI;
    const size_t rr = (size_t)R * R;
    const size_t need = (size_t)(N * rr + rr + (size_t)kPartials * rr + R) * 8;
    alto_status st = ensure_ws(&h->ws_sweep, &h->ws_sweep_bytes, need, s);
    if (st != ALTO_OK) return st;
    st = ensure_ws((void **)&h->ws_m, &h->ws_m_bytes, (size_t)maxI * R * 4, s);
    if (st != ALTO_OK) return st;
    size_t flag_bytes = h->ws_flags ? 256 : 0;
    st = ensure_ws((void **)&h->ws_flags, &flag_bytes, 256, s);
    if (st != ALTO_OK) return st;
    if (fdt == ALTO_BF16) {
        for (int m = 0; m < N; m++) {
            st = ensure_ws((void **)&h->ws_bf16[m], &h->ws_bf16_bytes[m], (size_t)h->info.dims[m] * R * 2, s);
            if (st != ALTO_OK) return st;
        }
    }
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(64), 0, s, h->ws_flags, (uint64_t)1, 0u);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

// Gram of mode m's factor into partials (and its BF16 shadow).
void gram_partials(alto_tensor *h, int m, int R, int fdt, float *const *factors, hipStream_t s) {
    const size_t rr = (size_t)R * R;
    double *partials = (double *)h->ws_sweep + h->info.nmodes * rr + rr;
    const uint64_t I = h->info.dims[m];
    launch_gram_rows<false>(R, partial_blocks(I), s, factors[m], nullptr, nullptr, I, partials);
    if (fdt == ALTO_BF16)
        hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(I * R, 256, 16384)), dim3(256), 0, s, factors[m], I * R,
                           h->ws_bf16[m]);
}

alto_status sweep_begin(alto_tensor *h, int rank, int fdt, float *const *factors, const double *lambda,
                        hipStream_t s) {
    alto_status st = sweep_setup(h, rank, fdt, factors, lambda, s);
    if (st != ALTO_OK) return st;
    const int N = h->info.nmodes;
    const int R = rank;
    const size_t rr = (size_t)R * R;
    double *grams = (double *)h->ws_sweep;
    double *partials = grams + N * rr + rr;
    for (int m = 0; m < N; m++) {
        gram_partials(h, m, R, fdt, factors, s);
        hipLaunchKernelGGL(k_gram_reduce, dim3(gram_reduce_blocks(R)), dim3(kThreads), 0, s, partials,
                           (int)partial_blocks(h->info.dims[m]), R, grams + m * rr);
    }
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

void sweep_factor_ptrs(const alto_tensor *h, int fdt, float *const *factors, const void **fptr) {
    for (int m = 0; m < h->info.nmodes; m++)
        fptr[m] = fdt == ALTO_BF16 ? (const void *)h->ws_bf16[m] : (const void *)factors[m];
}

alto_status sweep_pre(alto_tensor *h, int n, int rank, int rank_true, hipStream_t s) {
    const size_t rr = (size_t)rank * rank;
    double *grams = (double *)h->ws_sweep;
    double *W = grams + h->info.nmodes * rr;
    hipLaunchKernelGGL(k_als_prepare, dim3(1), dim3(kThreads), prepare_lds_bytes(rank), s, grams, h->info.nmodes, n, rank,
                       rank_true, W, h->ws_flags);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

alto_status sweep_post(alto_tensor *h, int n, int rank, int fdt, float *const *factors, double *lambda,
                       hipStream_t s) {
    const int R = rank;
    const size_t rr = (size_t)R * R;
    double *grams = (double *)h->ws_sweep;
    double *W = grams + h->info.nmodes * rr;
    double *partials = W + rr;
    double *lam_ws = partials + (size_t)kPartials * rr;
    const uint64_t I = h->info.dims[n];
    const unsigned P = partial_blocks(I);
    launch_gram_rows<true>(R, P, s, h->ws_m, W, factors[n], I, partials);
    hipLaunchKernelGGL(k_gram_reduce, dim3(gram_reduce_blocks(R)), dim3(kThreads), 0, s, partials, (int)P, R,
                       grams + n * rr);
    hipLaunchKernelGGL(k_als_finalize, dim3(1), dim3(kThreads), 0, s, grams + n * rr, R, lam_ws, lambda);
    hipLaunchKernelGGL(k_als_normalize, dim3(grid_for(I * R, 256, 16384)), dim3(256), 0, s, factors[n], I, R, lam_ws,
                       fdt == ALTO_BF16 ? h->ws_bf16[n] : nullptr);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

alto_status sweep_run(alto_tensor *h, int rank, int rank_true, int fdt, float *const *factors, double *lambda,
                      hipStream_t s) {
    alto_status st = sweep_begin(h, rank, fdt, factors, lambda, s);
    if (st != ALTO_OK) return st;
    const void *fptr[ALTO_MAX_MODES];
    sweep_factor_ptrs(h, fdt, factors, fptr);
    for (int n = 0; n < h->info.nmodes; n++) {
        st = sweep_pre(h, n, rank, rank_true, s);
        if (st != ALTO_OK) return st;
        alto_mttkrp_plan p;
        st = resolve_plan(h, n, rank, fdt, nullptr, &p);
        if (st != ALTO_OK) return st;
        st = run_mttkrp(h, n, rank, fdt, fptr, h->ws_m, p, s);
        if (st != ALTO_OK) return st;
        st = sweep_post(h, n, rank, fdt, factors, n == h->info.nmodes - 1 ? lambda : nullptr, s);
        if (st != ALTO_OK) return st;
    }
    return ALTO_OK;
}

// ---- batched sweeps (many tensors, interleaved mode by mode)

namespace {

// The host description of one batched sweep: the jobs, and the table of
// their per-mode R x R steps (section m: the jobs that have a mode m).
struct BatchedSweep {
    int count = 0, maxN = 0, maxR = 0;
    std::vector<alto_tensor *> hs;
    std::vector<int> ranks, fdts;
    std::vector<float *> facs;         // count x ALTO_MAX_MODES factor pointers
    std::vector<double *> lambdas;
    std::vector<const void *> fptr;    // count x ALTO_MAX_MODES gathered factors (BF16 shadows)
    std::vector<SweepJob> table;
    std::vector<size_t> sec;
    // per mode: the Gram launches, one per rank bucket (table range, bucket,
    // workgroups)
    struct GramRange {
        size_t b0;
        int nj, rb;
        unsigned blocks;
    };
    std::vector<std::vector<GramRange>> granges;
    unsigned nblk = 1, rblocks = 1;
};

// A job that fills the GPU by itself runs its own MTTKRP launch with its
// mode's plan (whole-mode LDS, rank tiles); the small ones share persistent
// launches.
bool runs_alone(const alto_tensor *h) { return h->info.nnz >= kBatchAloneNnz; }

// Such a job accumulates in FP32 or in one FP64 buffer (dims x rank doubles,
// which the serving footprint counts), never in per-XCD copies.
void batched_alone_accumulation(alto_mttkrp_plan *p) {
    if (p->accumulate == ALTO_ACC_XCD_F64 || p->accumulate == ALTO_ACC_XCD_F32) p->accumulate = ALTO_ACC_F64;
}

}  // namespace

}  // namespace alto

using namespace alto;

// A batched sweep prepared once: its device tables (the R x R step table and
// the planned MTTKRP groups of every mode) and the alone jobs' plans, so that
// a run only launches kernels.
struct alto_sweep_batch {
    static constexpr uint32_t kMagic = 0x53574250u;
    uint32_t magic = kMagic;
    int device = 0;
    BatchedSweep bs;
    std::vector<std::vector<std::pair<int, alto_mttkrp_plan>>> alone;  // per mode: (job, plan)
    std::vector<std::vector<GroupLaunch>> groups;                      // per mode
    std::vector<std::vector<size_t>> offs;                             // their blob offsets
    std::vector<char> host;                                            // the device tables' image
    void *dev = nullptr;
    hipStream_t last = nullptr;
    // each handle's workspaces when the tables were built (they point there)
    std::vector<std::array<const void *, 4 + ALTO_MAX_MODES>> ws;
};

namespace {

std::array<const void *, 4 + ALTO_MAX_MODES> ws_of(const alto_tensor *h) {
    std::array<const void *, 4 + ALTO_MAX_MODES> w{};
    w[0] = h->ws_sweep;
    w[1] = h->ws_m;
    w[2] = h->ws_flags;
    w[3] = h->ws_acc;
    for (int m = 0; m < h->info.nmodes; m++) w[4 + m] = h->ws_bf16[m];
    return w;
}

// Validation, workspaces and the step table of a batched sweep.
alto_status batched_sweep_setup(int count, const alto_handle *hs, const int *ranks, const int *fdts,
                                float *const *const *factors, double *const *lambdas, hipStream_t s,
                                BatchedSweep *bs) {
    if (!hs || !ranks || !fdts || !factors || !lambdas) return fail(ALTO_ERR_ARG, "NULL argument");
    bs->count = count;
    bs->hs.assign(hs, hs + count);
    bs->ranks.assign(ranks, ranks + count);
    bs->fdts.assign(fdts, fdts + count);
    bs->lambdas.assign(lambdas, lambdas + count);
    bs->facs.assign((size_t)count * ALTO_MAX_MODES, nullptr);
    for (int j = 0; j < count; j++) {
        if (!factors[j]) return fail(ALTO_ERR_ARG, "factors[" + std::to_string(j) + "] is NULL");
        alto_status st = sweep_setup(hs[j], ranks[j], fdts[j], factors[j], lambdas[j], s);
        if (st != ALTO_OK) return fail(st, "item " + std::to_string(j) + ": " + alto_last_error());
        bs->maxN = std::max(bs->maxN, hs[j]->info.nmodes);
        bs->maxR = std::max(bs->maxR, ranks[j]);
        for (int m = 0; m < hs[j]->info.nmodes; m++) bs->facs[(size_t)j * ALTO_MAX_MODES + m] = factors[j][m];
    }
    const int maxN = bs->maxN;
    bs->sec.assign(maxN + 1, 0);
    for (int m = 0; m < maxN; m++) {
        bs->sec[m] = bs->table.size();
        for (int j = 0; j < count; j++) {
            alto_tensor *h = hs[j];
            if (m >= h->info.nmodes) continue;
            const int R = ranks[j];
            const size_t rr = (size_t)R * R;
            double *grams = (double *)h->ws_sweep;
            double *W = grams + h->info.nmodes * rr;
            double *partials = W + rr;
            SweepJob jb;
            jb.grams = grams;
            jb.W = W;
            jb.flags = h->ws_flags;
            jb.partials = partials;
            jb.G = grams + m * rr;
            jb.lam_ws = partials + (size_t)kPartials * rr;
            jb.lam_out = m == h->info.nmodes - 1 ? lambdas[j] : nullptr;
            jb.A = factors[j][m];
            jb.shadow = fdts[j] == ALTO_BF16 ? h->ws_bf16[m] : nullptr;
            jb.M = h->ws_m;
            jb.I = h->info.dims[m];
            jb.N = h->info.nmodes;
            jb.n = m;
            jb.R = R;
            jb.P = (int)partial_blocks(jb.I);
            jb.blk0 = 0;
            bs->table.push_back(jb);
        }
        // the mode's jobs ordered by rank bucket: one Gram launch per bucket
        auto first = bs->table.begin() + bs->sec[m];
        std::stable_sort(first, bs->table.end(), [](const SweepJob &x, const SweepJob &y) {
            return rank_bucket(x.R) < rank_bucket(y.R);
        });
    }
    bs->sec[maxN] = bs->table.size();
    bs->granges.assign(maxN, {});
    for (int m = 0; m < maxN; m++) {
        for (size_t k = bs->sec[m]; k < bs->sec[m + 1];) {
            const int rb = rank_bucket(bs->table[k].R);
            BatchedSweep::GramRange g{k, 0, rb, 0};
            for (; k < bs->sec[m + 1] && rank_bucket(bs->table[k].R) == rb; k++) {
                bs->table[k].blk0 = g.blocks;
                g.blocks += (unsigned)bs->table[k].P;
                g.nj++;
            }
            bs->granges[m].push_back(g);
        }
    }
    // normalization grid (every workgroup takes part in every job): enough
    // workgroups for the largest factor
    uint64_t maxIR = 1;
    for (const SweepJob &jb : bs->table) maxIR = std::max<uint64_t>(maxIR, jb.I * (uint64_t)jb.R);
    bs->nblk = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(4096, (maxIR + 2047) / 2048));
    bs->rblocks = gram_reduce_blocks(bs->maxR);
    bs->fptr.assign((size_t)count * ALTO_MAX_MODES, nullptr);
    for (int j = 0; j < count; j++)
        sweep_factor_ptrs(hs[j], fdts[j], &bs->facs[(size_t)j * ALTO_MAX_MODES], &bs->fptr[(size_t)j * ALTO_MAX_MODES]);
    return ALTO_OK;
}

// The launch sequence of a batched sweep.  With a prepared batch `pb`, the
// MTTKRPs use its plans and device tables (kernel launches only); without,
// plans are resolved and the group tables uploaded now.
alto_status batched_sweep_launch(const BatchedSweep &bs, const SweepJob *dtab, const alto_sweep_batch *pb,
                                 const char *dbase, hipStream_t s) {
    const int count = bs.count;
    // Grams of every factor: the partials of mode m for every job, then one
    // reduction launch (each job's partial buffer is reused mode by mode)
    for (int m = 0; m < bs.maxN; m++) {
        for (const BatchedSweep::GramRange &g : bs.granges[m])
            launch_gram_rows_b<false>(g.rb, g.blocks, s, dtab + g.b0, g.nj);
        const unsigned nj = (unsigned)(bs.sec[m + 1] - bs.sec[m]);
        hipLaunchKernelGGL(k_gram_reduce_b, dim3(nj, bs.rblocks), dim3(kThreads), 0, s, dtab + bs.sec[m]);
    }
    ALTO_HIP(hipGetLastError());
    std::vector<alto_handle> bh;
    std::vector<int> bm, br, bf;
    std::vector<const void *const *> bfac;
    std::vector<float *> bout;
    for (int n = 0; n < bs.maxN; n++) {
        const unsigned nj = (unsigned)(bs.sec[n + 1] - bs.sec[n]);
        // V, Cholesky and solve operator of mode n for every job
        hipLaunchKernelGGL(k_als_prepare_b, dim3(nj), dim3(kThreads), prepare_lds_bytes(bs.maxR), s,
                           dtab + bs.sec[n]);
        ALTO_HIP(hipGetLastError());
        alto_status st = ALTO_OK;
        if (pb) {
            for (const auto &jp : pb->alone[n]) {
                const int j = jp.first;
                st = run_mttkrp(bs.hs[j], n, bs.ranks[j], bs.fdts[j], &bs.fptr[(size_t)j * ALTO_MAX_MODES],
                                bs.hs[j]->ws_m, jp.second, s);
                if (st != ALTO_OK) return st;
            }
            for (size_t k = 0; k < pb->groups[n].size(); k++) {
                st = launch_planned_group(pb->groups[n][k], dbase + pb->offs[n][k], s);
                if (st != ALTO_OK) return st;
            }
        } else {
            bh.clear(); bm.clear(); br.clear(); bf.clear(); bfac.clear(); bout.clear();
            for (int j = 0; j < count; j++) {
                if (n >= bs.hs[j]->info.nmodes) continue;
                if (runs_alone(bs.hs[j])) {
                    alto_mttkrp_plan p;
                    st = resolve_plan(bs.hs[j], n, bs.ranks[j], bs.fdts[j], nullptr, &p);
                    if (st != ALTO_OK) return st;
                    batched_alone_accumulation(&p);
                    st = run_mttkrp(bs.hs[j], n, bs.ranks[j], bs.fdts[j], &bs.fptr[(size_t)j * ALTO_MAX_MODES],
                                    bs.hs[j]->ws_m, p, s);
                    if (st != ALTO_OK) return st;
                    continue;
                }
                bh.push_back(bs.hs[j]);
                bm.push_back(n);
                br.push_back(bs.ranks[j]);
                bf.push_back(bs.fdts[j]);
                bfac.push_back(&bs.fptr[(size_t)j * ALTO_MAX_MODES]);
                bout.push_back(bs.hs[j]->ws_m);
            }
            // the MTTKRPs of mode n of every job in one persistent launch per
            // kernel variant
            st = bh.empty() ? ALTO_OK
                            : batched_run((int)bh.size(), bh.data(), bm.data(), br.data(), bf.data(), bfac.data(),
                                          bout.data(), s);
            if (st != ALTO_OK) return st;
        }
        // A = M W with the partial Grams of A (one launch per rank bucket),
        // then the Gram sums, lambda and normalization in one launch each
        for (const BatchedSweep::GramRange &g : bs.granges[n])
            launch_gram_rows_b<true>(g.rb, g.blocks, s, dtab + g.b0, g.nj);
        hipLaunchKernelGGL(k_gram_reduce_b, dim3(nj, bs.rblocks), dim3(kThreads), 0, s, dtab + bs.sec[n]);
        hipLaunchKernelGGL(k_als_finalize_b, dim3(nj), dim3(kThreads), 0, s, dtab + bs.sec[n]);
        hipLaunchKernelGGL(k_als_normalize_b, dim3(bs.nblk), dim3(256), 0, s, dtab + bs.sec[n], (int)nj);
        ALTO_HIP(hipGetLastError());
    }
    return ALTO_OK;
}

// Plans, reserved workspaces and device tables of a prepared batch.
alto_status batched_sweep_prepare(alto_sweep_batch *b, hipStream_t s) {
    BatchedSweep &bs = b->bs;
    const int maxN = bs.maxN;
    b->alone.assign(maxN, {});
    b->groups.assign(maxN, {});
    b->offs.assign(maxN, {});
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = align(bs.table.size() * sizeof(SweepJob));
    std::vector<alto_handle> bh;
    std::vector<int> bm, br, bf;
    std::vector<const void *const *> bfac;
    std::vector<float *> bout;
    for (int n = 0; n < maxN; n++) {
        bh.clear(); bm.clear(); br.clear(); bf.clear(); bfac.clear(); bout.clear();
        for (int j = 0; j < bs.count; j++) {
            alto_tensor *h = bs.hs[j];
            if (n >= h->info.nmodes) continue;
            if (runs_alone(h)) {
                alto_mttkrp_plan p;
                alto_status st = resolve_plan(h, n, bs.ranks[j], bs.fdts[j], nullptr, &p);
                if (st != ALTO_OK) return st;
                batched_alone_accumulation(&p);
                if (p.accumulate != ALTO_ACC_F32) {
                    // the accumulation buffer the run will use, allocated now
                    const bool f64 = p.accumulate == ALTO_ACC_F64 || p.accumulate == ALTO_ACC_XCD_F64;
                    const int copies = (p.accumulate == ALTO_ACC_XCD_F32 || p.accumulate == ALTO_ACC_XCD_F64) ? kXcdCopies : 1;
                    st = ensure_ws(&h->ws_acc, &h->ws_acc_bytes,
                                   h->info.dims[n] * (size_t)bs.ranks[j] * copies * (f64 ? 8 : 4), s);
                    if (st != ALTO_OK) return st;
                }
                b->alone[n].push_back({j, p});
                continue;
            }
            bh.push_back(h);
            bm.push_back(n);
            br.push_back(bs.ranks[j]);
            bf.push_back(bs.fdts[j]);
            bfac.push_back(&bs.fptr[(size_t)j * ALTO_MAX_MODES]);
            bout.push_back(h->ws_m);
        }
        if (bh.empty()) continue;
        alto_status st = batched_plan((int)bh.size(), bh.data(), bm.data(), br.data(), bf.data(), bfac.data(),
                                      bout.data(), s, &b->groups[n]);
        if (st != ALTO_OK) return st;
        for (const GroupLaunch &gl : b->groups[n]) {
            b->offs[n].push_back(off);
            off += align(gl.blob_bytes());
        }
    }
    b->host.assign(off, 0);
    memcpy(b->host.data(), bs.table.data(), bs.table.size() * sizeof(SweepJob));
    for (int n = 0; n < maxN; n++)
        for (size_t k = 0; k < b->groups[n].size(); k++) b->groups[n][k].write_blob(b->host.data() + b->offs[n][k]);
    if (dev_alloc(&b->dev, off) != hipSuccess) return fail(ALTO_ERR_OOM, "sweep batch table allocation failed");
    b->last = s;
    ALTO_HIP(hipMemcpyAsync(b->dev, b->host.data(), off, hipMemcpyHostToDevice, s));
    ALTO_HIP(hipStreamSynchronize(s));
    b->ws.clear();
    for (int j = 0; j < bs.count; j++) b->ws.push_back(ws_of(bs.hs[j]));
    return ALTO_OK;
}

// The tables point into the handles' workspaces: a run is refused once any
// of them was reallocated (by a larger call on the same handle).
alto_status batched_sweep_check(const alto_sweep_batch *b) {
    for (int j = 0; j < b->bs.count; j++) {
        ALTO_CHECK_HANDLE(b->bs.hs[j]);
        if (ws_of(b->bs.hs[j]) != b->ws[j])
            return fail(ALTO_ERR_STATE, "sweep batch item " + std::to_string(j) +
                                            ": the handle's workspace changed since the batch was created");
    }
    return ALTO_OK;
}

}  // namespace

extern "C" {

alto_status cpd_als_sweep_ex(alto_handle h, int rank, alto_dtype fdt, float *const *factors, double *lambda,
                             void *stream) {
    ALTO_CHECK_HANDLE(h);
    hipStream_t s = (hipStream_t)stream;
    if (rank % 4 == 0 || rank < 1) return sweep_run(h, rank, rank, fdt, factors, lambda, s);
    // a rank that is not a multiple of 4: sweep zero-padded copies
    if (rank > kMaxSweepRank) return fail(ALTO_ERR_ARG, "sweep rank must be in 1..64");
    if (!factors || !lambda) return fail(ALTO_ERR_ARG, "factors/lambda is NULL");
    const int R4 = padded_rank(rank);
    void *pf[ALTO_MAX_MODES];
    alto_status st = pad_factors(h, rank, ALTO_F32, (const void *const *)factors, -1, pf, s);
    if (st != ALTO_OK) return st;
    st = ensure_ws((void **)&h->ws_lampad, &h->ws_lampad_bytes, (size_t)R4 * sizeof(double), s);
    if (st != ALTO_OK) return st;
    st = sweep_run(h, R4, rank, fdt, (float *const *)pf, h->ws_lampad, s);
    if (st != ALTO_OK) return st;
    for (int m = 0; m < h->info.nmodes; m++) launch_copy_cols(pf[m], R4, factors[m], rank, h->info.dims[m], 4, s);
    ALTO_HIP(hipMemcpyAsync(lambda, h->ws_lampad, (size_t)rank * sizeof(double), hipMemcpyDeviceToDevice, s));
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

alto_status cpd_als_sweep_batched(int count, const alto_handle *hs, const int *ranks, const int *fdts,
                                  float *const *const *factors, double *const *lambdas, void *stream) {
    if (count < 0) return fail(ALTO_ERR_ARG, "count < 0");
    if (count == 0) return ALTO_OK;
    hipStream_t s = (hipStream_t)stream;
    BatchedSweep bs;
    alto_status st = batched_sweep_setup(count, hs, ranks, fdts, factors, lambdas, s, &bs);
    if (st != ALTO_OK) return st;
    SweepJob *dtab = nullptr;
    st = upload_sweep_jobs(bs.table, s, &dtab);
    if (st != ALTO_OK) return st;
    return batched_sweep_launch(bs, dtab, nullptr, nullptr, s);
}

alto_status alto_sweep_batch_create(int count, const alto_handle *hs, const int *ranks, const int *fdts,
                                    float *const *const *factors, double *const *lambdas, void *stream,
                                    alto_sweep_batch_t *out) {
    if (!out) return fail(ALTO_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1) return fail(ALTO_ERR_ARG, "count must be at least 1");
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<alto_sweep_batch> b(new alto_sweep_batch());
    alto_status st = batched_sweep_setup(count, hs, ranks, fdts, factors, lambdas, s, &b->bs);
    if (st != ALTO_OK) return st;
    ALTO_HIP(hipGetDevice(&b->device));
    for (int j = 0; j < count; j++)
        if (hs[j]->device != b->device) return fail(ALTO_ERR_ARG, "every handle must be on the current device");
    st = batched_sweep_prepare(b.get(), s);
    if (st != ALTO_OK) return st;
    *out = b.release();
    return ALTO_OK;
}

alto_status alto_sweep_batch_run(alto_sweep_batch_t b, void *stream) {
    if (!b || b->magic != alto_sweep_batch::kMagic) return fail(ALTO_ERR_STATE, "not a sweep batch");
    hipStream_t s = (hipStream_t)stream;
    int dev = -1;
    ALTO_HIP(hipGetDevice(&dev));
    if (dev != b->device) return fail(ALTO_ERR_ARG, "the batch's device is not the current device");
    alto_status st = batched_sweep_check(b);
    if (st != ALTO_OK) return st;
    for (int j = 0; j < b->bs.count; j++) {
        b->bs.hs[j]->stream = s;
        hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(64), 0, s, b->bs.hs[j]->ws_flags, (uint64_t)1, 0u);
    }
    ALTO_HIP(hipGetLastError());
    b->last = s;
    return batched_sweep_launch(b->bs, (const SweepJob *)b->dev, b, (const char *)b->dev, s);
}

alto_status alto_sweep_batch_destroy(alto_sweep_batch_t b) {
    if (!b) return ALTO_OK;
    if (b->magic != alto_sweep_batch::kMagic) return fail(ALTO_ERR_STATE, "not a sweep batch");
    b->magic = 0;
    if (b->dev) dev_free_after(b->dev, b->last);
    delete b;
    return ALTO_OK;
}

alto_status cpd_als_sweep(alto_handle h, int rank, float *const *factors, double *lambda, void *stream) {
    return cpd_als_sweep_ex(h, rank, ALTO_F32, factors, lambda, stream);
}

alto_status alto_sweep_flags(alto_handle h, void *stream, uint32_t *flags) {
    ALTO_CHECK_HANDLE(h);
    if (!flags) return fail(ALTO_ERR_ARG, "flags is NULL");
    *flags = 0;
    if (!h->ws_flags) return ALTO_OK;
    hipStream_t s = (hipStream_t)stream;
    ALTO_HIP(hipMemcpyAsync(flags, h->ws_flags, 4, hipMemcpyDeviceToHost, s));
    ALTO_HIP(hipStreamSynchronize(s));
    return *flags ? ALTO_ERR_NOT_SPD : ALTO_OK;
}

}  // extern "C"
