// ALTO format generation on the GPU (Sec. "ALTO Tensor Generation" and
// "Workload Partitioning and Scheduling" of the paper):
//   1. linearization: every nonzero's coordinates are deposited into the
//      bit positions of its mode's mask (bit-level gather);
//   2. ordering: a stable least-significant-digit radix sort of
//      (index, value) pairs over the ceil(B/8) bytes that carry index bits;
//   3. partitioning: nnz-balanced line segments and their mode intervals.
#include <string.h>

#include <algorithm>
#include <string>

#include "alto_internal.h"
#include "device_util.h"
#include "memory.h"

namespace alto {
namespace {

// ------------------------------------------------------------ encode

struct EncodeArgs {
    LinePlan lp;
    const int64_t *coords[ALTO_MAX_MODES];
    uint64_t dims[ALTO_MAX_MODES];
    const float *vals_in;
    uint64_t *keys;
    float *vals;
    uint64_t n;
    unsigned long long *first_bad;
};

template <int WORDS>
__global__ __launch_bounds__(256) void k_encode(const EncodeArgs a) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        uint64_t lo = 0, hi = 0;
        bool ok = true;
        // modes in a rolled loop: the masks are fetched per mode into scalar
        // registers instead of holding all of them at once
#pragma unroll 1
        for (int m = 0; m < a.lp.nmodes; m++) {
            const int64_t c = a.coords[m][i];
            ok = ok && c >= 0 && (uint64_t)c < a.dims[m];
            const uint64_t cu = (uint64_t)c;
            lo |= deposit_word(cu, a.lp.mode[m].w[0]);
            if (WORDS == 2) hi |= deposit_word(cu >> a.lp.mode[m].lo_bits, a.lp.mode[m].w[1]);
        }
        if (!ok) atomicMin(a.first_bad, (unsigned long long)i);
        a.keys[i * WORDS] = lo;
        if (WORDS == 2) a.keys[i * WORDS + 1] = hi;
        a.vals[i] = a.vals_in[i];
    }
}

// ------------------------------------------------------------ radix sort

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;

template <int WORDS>
struct RsCfg;
template <>
struct RsCfg<1> {
    static constexpr int IPT = 12;  // 8 and 16 measured slower on 1e8 keys
};
template <>
struct RsCfg<2> {
    static constexpr int IPT = 8;
};

template <int WORDS>
__device__ inline uint32_t digit_at(const uint64_t *k, int shift) {
    const uint64_t w = (WORDS == 2 && shift >= 64) ? k[1] : k[0];
    return (uint32_t)(w >> (shift & 63)) & 0xFFu;
}

// Workgroups are dealt to the 8 XCDs round-robin.  Renumbering them so that
// each XCD takes a contiguous run of tiles puts the blocks whose digit counts
// and offsets share a cache line (adjacent b of counts[d * nblocks + b]) in
// the same L2.  The map is a bijection on 0..nblocks-1 whatever the placement.
__device__ inline uint32_t xcd_tile(uint32_t bid, uint32_t nblocks) {
    const uint32_t x = bid & 7u, q = nblocks >> 3, r = nblocks & 7u;
    return x * q + min(x, r) + (bid >> 3);
}

// Per-block digit counts, stored digit-major: counts[d * nblocks + b].
template <int WORDS>
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t *__restrict__ keys, uint64_t n, int shift,
                                                        uint32_t *__restrict__ counts, uint32_t nblocks) {
    constexpr int TILE = RS_THREADS * RsCfg<WORDS>::IPT;
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t blk = xcd_tile(blockIdx.x, nblocks);
    const uint64_t base = (uint64_t)blk * TILE;
    const int lane = lane_id();
    // all of the thread's key loads are issued before the first is used
    uint32_t dg[RsCfg<WORDS>::IPT];
#pragma unroll
    for (int j = 0; j < RsCfg<WORDS>::IPT; j++) {
        const uint64_t i = base + (uint64_t)j * RS_THREADS + threadIdx.x;
        dg[j] = i < n ? digit_at<WORDS>(keys + i * WORDS, shift) : 0u;
    }
#pragma unroll
    for (int j = 0; j < RsCfg<WORDS>::IPT; j++) {
        const uint64_t i = base + (uint64_t)j * RS_THREADS + threadIdx.x;
        const bool valid = i < n;
        const uint32_t d = dg[j];
        const uint64_t act = __ballot(valid);
        const uint64_t peers = match_byte(d, act);
        // one update per distinct digit of the wave (Zipf inputs repeat keys)
        if (valid && (peers & ((uint64_t(1) << lane) - 1)) == 0) atomicAdd(&hist[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    counts[(uint64_t)threadIdx.x * nblocks + blk] = hist[threadIdx.x];
}

constexpr int SC_THREADS = 256;
constexpr int SC_IPT = 16;
constexpr int SC_TILE = SC_THREADS * SC_IPT;

__global__ __launch_bounds__(SC_THREADS) void k_scan_reduce(const uint32_t *__restrict__ in, uint64_t n,
                                                            uint64_t *__restrict__ partial) {
    __shared__ uint64_t sc[SC_THREADS / 64];
    const uint64_t base = (uint64_t)blockIdx.x * SC_TILE;
    uint64_t s = 0;
    for (int j = 0; j < SC_IPT; j++) {
        const uint64_t i = base + (uint64_t)j * SC_THREADS + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint64_t tot;
    block_exclusive_scan<uint64_t>(s, sc, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_top(uint64_t *partial, uint64_t np) {
    __shared__ uint64_t sc[SC_THREADS / 64];
    uint64_t carry = 0;
    for (uint64_t c = 0; c < np; c += SC_THREADS) {
        const uint64_t i = c + threadIdx.x;
        const uint64_t v = i < np ? partial[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_exclusive_scan<uint64_t>(v, sc, &tot);
        if (i < np) partial[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_apply(const uint32_t *__restrict__ in, uint64_t n,
                                                           const uint64_t *__restrict__ partial,
                                                           uint64_t *__restrict__ out) {
    __shared__ uint64_t sc[SC_THREADS / 64];
    const uint64_t base = (uint64_t)blockIdx.x * SC_TILE + (uint64_t)threadIdx.x * SC_IPT;
    uint32_t v[SC_IPT];
    uint64_t s = 0;
    for (int j = 0; j < SC_IPT; j++) {
        v[j] = (base + j < n) ? in[base + j] : 0u;
        s += v[j];
    }
    uint64_t tot;
    uint64_t run = block_exclusive_scan<uint64_t>(s, sc, &tot) + partial[blockIdx.x];
    for (int j = 0; j < SC_IPT; j++) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
}

// Stable scatter of one digit pass.  Wave w of block b owns the contiguous
// items [b*TILE + w*64*IPT, ... + 64*IPT); within a wave, iteration j covers
// 64 consecutive items, so (wave, iteration, lane) is the input order.  Each
// item's rank among equal digits is its wave-local running count (kept per
// wave in LDS) plus the counts of earlier waves; items are staged in LDS in
// block-sorted order and written out in runs per digit.
template <int WORDS>
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint64_t *__restrict__ keys_in,
                                                           const float *__restrict__ vals_in,
                                                           uint64_t *__restrict__ keys_out,
                                                           float *__restrict__ vals_out, uint64_t n, int shift,
                                                           const uint64_t *__restrict__ offsets, uint32_t nblocks) {
    constexpr int IPT = RsCfg<WORDS>::IPT;
    constexpr int TILE = RS_THREADS * IPT;
    __shared__ uint32_t wcnt[RS_WAVES][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint64_t goff[256];
    __shared__ uint32_t sc[RS_THREADS / 64];
    __shared__ uint64_t skeys[TILE * WORDS];
    __shared__ float svals[TILE];

    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    for (int i = tid; i < RS_WAVES * 256; i += RS_THREADS) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    const uint32_t blk = xcd_tile(blockIdx.x, nblocks);
    const uint64_t tbase = (uint64_t)blk * TILE;
    uint64_t kw[IPT][WORDS];
    float kv[IPT];
    uint32_t loc[IPT];
    // all of the thread's loads are issued before the ranking below uses them
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        const uint64_t i = tbase + (uint64_t)w * 64 * IPT + (uint64_t)j * 64 + lane;
        const bool valid = i < n;
#pragma unroll
        for (int q = 0; q < WORDS; q++) kw[j][q] = valid ? keys_in[i * WORDS + q] : 0;
        kv[j] = valid ? vals_in[i] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        const uint64_t i = tbase + (uint64_t)w * 64 * IPT + (uint64_t)j * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = valid ? digit_at<WORDS>(kw[j], shift) : 0u;
        const uint64_t act = __ballot(valid);
        const uint64_t peers = match_byte(d, act);
        const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        uint32_t basec = 0;
        if (valid) basec = wcnt[w][d];
        // the highest lane of each digit group advances the wave's counter;
        // LDS operations of one wave complete in issue order, so the next
        // iteration's reads see this write
        if (valid && (peers >> lane) == 1u) wcnt[w][d] = basec + (uint32_t)__popcll(peers);
        loc[j] = basec + rank;
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, then over digits
    {
        const int d = tid;  // RS_THREADS == 256 digits
        uint32_t run = 0;
        for (int k = 0; k < RS_WAVES; k++) {
            const uint32_t c = wcnt[k][d];
            wcnt[k][d] = run;
            run += c;
        }
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<uint32_t>(run, sc, &tot);
        dstart[d] = ex;
        goff[d] = offsets[(uint64_t)d * nblocks + blk];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        const uint64_t i = tbase + (uint64_t)w * 64 * IPT + (uint64_t)j * 64 + lane;
        if (i < n) {
            const uint32_t d = digit_at<WORDS>(kw[j], shift);
            const uint32_t p = dstart[d] + wcnt[w][d] + loc[j];
            if (p < (uint32_t)TILE) {  // always true; keeps a logic error from touching foreign LDS
#pragma unroll
                for (int q = 0; q < WORDS; q++) skeys[p * WORDS + q] = kw[j][q];
                svals[p] = kv[j];
            }
        }
    }
    __syncthreads();
    const uint32_t tile_n = (uint32_t)((n - tbase) < (uint64_t)TILE ? (n - tbase) : (uint64_t)TILE);
    for (uint32_t p = tid; p < tile_n; p += RS_THREADS) {
        uint64_t k[WORDS];
#pragma unroll
        for (int q = 0; q < WORDS; q++) k[q] = skeys[p * WORDS + q];
        const uint32_t d = digit_at<WORDS>(k, shift);
        const uint64_t dst = goff[d] + (p - dstart[d]);
        if (dst < n) {  // always true; keeps a logic error from writing out of bounds
#pragma unroll
            for (int q = 0; q < WORDS; q++) keys_out[dst * WORDS + q] = k[q];
            vals_out[dst] = svals[p];
        }
    }
}

// ------------------------------------------------------------ partition / decode

constexpr int kPartChunk = 8;

// A mode's bits of an index, as a (hi, lo) pair ordered like the coordinate:
// mask extraction keeps the relative order of the kept bits, so among indices
// masked to one mode the smallest masked value holds the smallest coordinate
// (and likewise the largest).  Min and max are therefore taken on masked
// indices and only the two results are decoded.
struct PartKey {
    uint64_t hi, lo;
};

__device__ inline bool part_less(const PartKey &x, const PartKey &y) {
    return x.hi < y.hi || (x.hi == y.hi && x.lo < y.lo);
}

__device__ inline uint64_t shfl_xor64(uint64_t v, int o) {
    const int a = __shfl_xor((int)(uint32_t)v, o, 64);
    const int b = __shfl_xor((int)(uint32_t)(v >> 32), o, 64);
    return (uint64_t)(uint32_t)a | ((uint64_t)(uint32_t)b << 32);
}

template <int WORDS>
__device__ inline PartKey part_shfl(const PartKey &k, int o) {
    return PartKey{WORDS == 2 ? shfl_xor64(k.hi, o) : 0, shfl_xor64(k.lo, o)};
}

// Segments l = 0..nseg-1 (a grid-stride loop of workgroups): start offset and
// the closed interval of every mode's coordinates.  Per mode, the minimum and
// maximum masked index are reduced across each wave with shuffles, then across
// the 4 waves in LDS, and decoded once.
template <int WORDS>
__global__ __launch_bounds__(256) void k_partition(const LinePlan lp, const uint64_t *__restrict__ keys, uint64_t n,
                                                   uint64_t nseg, int64_t *__restrict__ starts,
                                                   uint64_t *__restrict__ iv) {
    __shared__ PartKey wmin[4][ALTO_MAX_MODES], wmax[4][ALTO_MAX_MODES];
    const int N = lp.nmodes;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const uint64_t q = n / nseg, r = n % nseg;
    for (uint64_t l = blockIdx.x; l < nseg; l += gridDim.x) {
        const uint64_t a = l * q + (l * r) / nseg;
        const uint64_t b = (l + 1) * q + ((l + 1) * r) / nseg;
        if (threadIdx.x == 0) {
            starts[l] = (int64_t)a;
            if (l == nseg - 1) starts[nseg] = (int64_t)n;
        }
        PartKey mn[ALTO_MAX_MODES], mx[ALTO_MAX_MODES];
#pragma unroll
        for (int m = 0; m < ALTO_MAX_MODES; m++) {
            mn[m] = PartKey{~uint64_t(0), ~uint64_t(0)};
            mx[m] = PartKey{0, 0};
        }
        // chunks of kPartChunk keys per thread, loaded before they are used
        for (uint64_t x0 = a; x0 < b; x0 += (uint64_t)kPartChunk * blockDim.x) {
            uint64_t lo[kPartChunk], hi[kPartChunk];
            bool ok[kPartChunk];
#pragma unroll
            for (int j = 0; j < kPartChunk; j++) {
                const uint64_t x = x0 + (uint64_t)j * blockDim.x + threadIdx.x;
                ok[j] = x < b;
                lo[j] = ok[j] ? keys[x * WORDS] : 0;
                hi[j] = (WORDS == 2 && ok[j]) ? keys[x * WORDS + 1] : 0;
            }
#pragma unroll
            for (int j = 0; j < kPartChunk; j++) {
                if (!ok[j]) continue;
#pragma unroll
                for (int m = 0; m < ALTO_MAX_MODES; m++) {
                    if (m < N) {
                        const PartKey k{WORDS == 2 ? hi[j] & lp.mode[m].w[1].mask : 0, lo[j] & lp.mode[m].w[0].mask};
                        if (part_less(k, mn[m])) mn[m] = k;
                        if (part_less(mx[m], k)) mx[m] = k;
                    }
                }
            }
        }
#pragma unroll
        for (int m = 0; m < ALTO_MAX_MODES; m++) {
            if (m < N) {
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const PartKey u = part_shfl<WORDS>(mn[m], o), v = part_shfl<WORDS>(mx[m], o);
                    if (part_less(u, mn[m])) mn[m] = u;
                    if (part_less(mx[m], v)) mx[m] = v;
                }
                if (lane == 0) {
                    wmin[w][m] = mn[m];
                    wmax[w][m] = mx[m];
                }
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < N) {
            const int m = threadIdx.x;
            PartKey a0 = wmin[0][m], a1 = wmax[0][m];
            for (int k = 1; k < (int)(blockDim.x >> 6); k++) {
                if (part_less(wmin[k][m], a0)) a0 = wmin[k][m];
                if (part_less(a1, wmax[k][m])) a1 = wmax[k][m];
            }
            uint64_t *o = iv + (l * N + m) * 2;
            if (a == b) {  // empty segment: start > end
                o[0] = ~uint64_t(0);
                o[1] = 0;
            } else {
                o[0] = extract_mode<WORDS>(lp.mode[m], a0.lo, a0.hi);
                o[1] = extract_mode<WORDS>(lp.mode[m], a1.lo, a1.hi);
            }
        }
        __syncthreads();
    }
}

template <int WORDS>
__global__ __launch_bounds__(256) void k_decode(const LinePlan lp, const uint64_t *__restrict__ keys, uint64_t count,
                                                int64_t *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < count; x += stride) {
        const uint64_t lo = keys[x * WORDS];
        const uint64_t hi = WORDS == 2 ? keys[x * WORDS + 1] : 0;
#pragma unroll 1
        for (int m = 0; m < lp.nmodes; m++) out[(uint64_t)m * count + x] = extract_mode<WORDS>(lp.mode[m], lo, hi);
    }
}

// ------------------------------------------------------------ host side

struct Buf {
    void *p = nullptr;
    ~Buf() { dev_free(p); }
    hipError_t alloc(size_t b) { return dev_alloc(&p, b); }
};

template <int WORDS>
hipError_t radix_sort(uint64_t *&keys, float *&vals, uint64_t *&keys_alt, float *&vals_alt, uint64_t n, int bits,
                      hipStream_t s, uint32_t *counts, uint64_t *offsets, uint64_t *partials) {
    if (n <= 1 || bits == 0) return hipSuccess;
    constexpr int TILE = RS_THREADS * RsCfg<WORDS>::IPT;
    const uint32_t nblocks = (uint32_t)((n + TILE - 1) / TILE);
    const uint64_t ncounts = (uint64_t)256 * nblocks;
    const uint32_t npart = (uint32_t)((ncounts + SC_TILE - 1) / SC_TILE);
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist<WORDS>, dim3(nblocks), dim3(RS_THREADS), 0, s, keys, n, shift, counts, nblocks);
        hipLaunchKernelGGL(k_scan_reduce, dim3(npart), dim3(SC_THREADS), 0, s, counts, ncounts, partials);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SC_THREADS), 0, s, partials, (uint64_t)npart);
        hipLaunchKernelGGL(k_scan_apply, dim3(npart), dim3(SC_THREADS), 0, s, counts, ncounts, partials, offsets);
        hipLaunchKernelGGL(k_rs_scatter<WORDS>, dim3(nblocks), dim3(RS_THREADS), 0, s, keys, vals, keys_alt, vals_alt,
                           n, shift, offsets, nblocks);
        std::swap(keys, keys_alt);
        std::swap(vals, vals_alt);
    }
    return hipGetLastError();
}

template <int WORDS>
uint32_t sort_tile() {
    return RS_THREADS * RsCfg<WORDS>::IPT;
}

}  // namespace
}  // namespace alto

using namespace alto;

extern "C" {

alto_status alto_build(int nmodes, const uint64_t *dims, uint64_t nnz, const int64_t *const *coords,
                       const float *vals, void *stream, alto_handle *out) {
    if (!out) return fail(ALTO_ERR_ARG, "out is NULL");
    *out = nullptr;
    alto_info_t info;
    LinePlan lp;
    alto_status st = make_plan(nmodes, dims, &info, &lp);
    if (st != ALTO_OK) return st;
    if (nnz >= (uint64_t(1) << 40)) return fail(ALTO_ERR_ARG, "nnz must be below 2^40");
    if (nnz > 0) {
        if (!coords || !vals) return fail(ALTO_ERR_ARG, "coords/vals is NULL");
        for (int n = 0; n < nmodes; n++)
            if (!coords[n]) return fail(ALTO_ERR_ARG, "coords[" + std::to_string(n) + "] is NULL");
    }
    hipStream_t s = (hipStream_t)stream;
    const int W = info.index_words;

    alto_tensor *h = new alto_tensor();
    memset(h, 0, sizeof(*h));
    h->magic = kHandleMagic;
    ALTO_HIP(hipGetDevice(&h->device));
    h->stream = s;
    info.nnz = nnz;
    h->info = info;
    h->lp = lp;

    auto cleanup = [&](alto_status code, const std::string &msg) {
        dev_free(h->keys);
        dev_free(h->vals);
        h->magic = 0;
        delete h;
        return fail(code, msg);
    };

    const size_t kbytes = (size_t)nnz * W * 8, vbytes = (size_t)nnz * 4;
    if (dev_alloc((void **)&h->keys, kbytes) != hipSuccess || dev_alloc((void **)&h->vals, vbytes) != hipSuccess)
        return cleanup(ALTO_ERR_OOM, "device allocation of the ALTO tensor failed");
    if (nnz == 0) {
        h->info.device_bytes = 0;
        *out = h;
        return ALTO_OK;
    }
    Buf kalt, valt, bad, counts, offsets, partials;
    const uint32_t tile = W == 2 ? sort_tile<2>() : sort_tile<1>();
    const uint64_t nblocks = (nnz + tile - 1) / tile;
    const uint64_t ncounts = 256 * nblocks;
    const uint64_t npart = (ncounts + SC_TILE - 1) / SC_TILE;
    if (kalt.alloc(kbytes) != hipSuccess || valt.alloc(vbytes) != hipSuccess || bad.alloc(8) != hipSuccess ||
        counts.alloc(ncounts * 4) != hipSuccess || offsets.alloc(ncounts * 8) != hipSuccess ||
        partials.alloc(npart * 8) != hipSuccess)
        return cleanup(ALTO_ERR_OOM, "device allocation of build scratch failed");

    EncodeArgs ea;
    memset(&ea, 0, sizeof(ea));
    ea.lp = lp;
    for (int n = 0; n < nmodes; n++) {
        ea.coords[n] = coords[n];
        ea.dims[n] = dims[n];
    }
    ea.vals_in = vals;
    ea.keys = h->keys;
    ea.vals = h->vals;
    ea.n = nnz;
    ea.first_bad = (unsigned long long *)bad.p;
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (unsigned long long *)bad.p, (uint64_t)1,
                       ~0ull);
    const unsigned grid = grid_for(nnz, 256, 8192);
    if (W == 2) hipLaunchKernelGGL(k_encode<2>, dim3(grid), dim3(256), 0, s, ea);
    else hipLaunchKernelGGL(k_encode<1>, dim3(grid), dim3(256), 0, s, ea);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cleanup(ALTO_ERR_HIP, std::string("encode launch: ") + hipGetErrorString(e));

    uint64_t *k0 = h->keys, *k1 = (uint64_t *)kalt.p;
    float *v0 = h->vals, *v1 = (float *)valt.p;
    e = W == 2 ? radix_sort<2>(k0, v0, k1, v1, nnz, info.index_bits, s, (uint32_t *)counts.p,
                               (uint64_t *)offsets.p, (uint64_t *)partials.p)
               : radix_sort<1>(k0, v0, k1, v1, nnz, info.index_bits, s, (uint32_t *)counts.p,
                               (uint64_t *)offsets.p, (uint64_t *)partials.p);
    if (e != hipSuccess) return cleanup(ALTO_ERR_HIP, std::string("radix sort launch: ") + hipGetErrorString(e));
    unsigned long long first_bad = 0;
    e = hipMemcpyAsync(&first_bad, bad.p, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cleanup(ALTO_ERR_HIP, std::string("build: ") + hipGetErrorString(e));
    // the sorted data may have ended in the scratch buffers: keep those
    if (k0 != h->keys) {
        kalt.p = h->keys;
        h->keys = k0;
    }
    if (v0 != h->vals) {
        valt.p = h->vals;
        h->vals = v0;
    }
    if (first_bad != ~0ull)
        return cleanup(ALTO_ERR_COORD_RANGE,
                       "coordinate out of range at nonzero " + std::to_string((unsigned long long)first_bad));
    h->info.device_bytes = dev_size(h->keys) + dev_size(h->vals);
    *out = h;
    return ALTO_OK;
}

alto_status alto_info(alto_handle h, alto_info_t *out) {
    ALTO_CHECK_HANDLE(h);
    if (!out) return fail(ALTO_ERR_ARG, "out is NULL");
    size_t ws = dev_size(h->ws_acc) + dev_size(h->ws_sweep) + dev_size(h->ws_m) + dev_size(h->ws_flags) +
                dev_size(h->ws_fit) + dev_size(h->ws_pad_out) + dev_size(h->ws_lampad);
    for (int n = 0; n < ALTO_MAX_MODES; n++) ws += dev_size(h->ws_pad[n]);
    for (int n = 0; n < ALTO_MAX_MODES; n++) ws += dev_size(h->ws_bf16[n]);
    h->info.device_bytes = dev_size(h->keys) + dev_size(h->vals) + ws;
    *out = h->info;
    return ALTO_OK;
}

alto_status alto_export(alto_handle h, uint64_t *keys_out, float *vals_out, void *stream) {
    ALTO_CHECK_HANDLE(h);
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    const uint64_t n = h->info.nnz;
    if (n == 0) return ALTO_OK;
    if (keys_out)
        ALTO_HIP(hipMemcpyAsync(keys_out, h->keys, n * h->info.index_words * 8, hipMemcpyDeviceToDevice, s));
    if (vals_out) ALTO_HIP(hipMemcpyAsync(vals_out, h->vals, n * 4, hipMemcpyDeviceToDevice, s));
    return ALTO_OK;
}

alto_status alto_decode(alto_handle h, uint64_t count, const uint64_t *keys, int64_t *coords_out, void *stream) {
    ALTO_CHECK_HANDLE(h);
    if (count == 0) return ALTO_OK;
    if (!keys || !coords_out) return fail(ALTO_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    const unsigned grid = grid_for(count, 256, 8192);
    if (h->info.index_words == 2) hipLaunchKernelGGL(k_decode<2>, dim3(grid), dim3(256), 0, s, h->lp, keys, count, coords_out);
    else hipLaunchKernelGGL(k_decode<1>, dim3(grid), dim3(256), 0, s, h->lp, keys, count, coords_out);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

alto_status alto_partition(alto_handle h, int64_t nseg, int64_t *starts_out, uint64_t *intervals_out, void *stream) {
    ALTO_CHECK_HANDLE(h);
    if (nseg < 1 || (uint64_t)nseg > (uint64_t(1) << 32)) return fail(ALTO_ERR_ARG, "nseg must be in 1..2^32");
    if (!starts_out || !intervals_out) return fail(ALTO_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    const unsigned grid = (unsigned)std::min<int64_t>(nseg, 65536);
    if (h->info.index_words == 2)
        hipLaunchKernelGGL(k_partition<2>, dim3(grid), dim3(256), 0, s, h->lp, h->keys, h->info.nnz, (uint64_t)nseg,
                           starts_out, intervals_out);
    else
        hipLaunchKernelGGL(k_partition<1>, dim3(grid), dim3(256), 0, s, h->lp, h->keys, h->info.nnz, (uint64_t)nseg,
                           starts_out, intervals_out);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

alto_status alto_free(alto_handle h) {
    ALTO_CHECK_HANDLE(h);
    // buffers go back to the cache behind the work already enqueued on the
    // handle's last stream; nothing waits here
    const hipStream_t s = h->stream;
    dev_free_after(h->keys, s);
    dev_free_after(h->vals, s);
    dev_free_after(h->ws_acc, s);
    dev_free_after(h->ws_sweep, s);
    dev_free_after(h->ws_m, s);
    dev_free_after(h->ws_flags, s);
    dev_free_after(h->ws_fit, s);
    dev_free_after(h->ws_pad_out, s);
    dev_free_after(h->ws_lampad, s);
    for (int n = 0; n < ALTO_MAX_MODES; n++) dev_free_after(h->ws_pad[n], s);
    for (int n = 0; n < ALTO_MAX_MODES; n++) dev_free_after(h->ws_bf16[n], s);
    for (int n = 0; n < ALTO_MAX_MODES; n++) dev_free_after(h->ws_apr_phi[n], s);
    dev_free_after(h->ws_apr_b, s);
    dev_free_after(h->ws_apr_red, s);
    dev_free_after(h->ws_apr_pi, s);
    h->magic = 0;
    delete h;
    return ALTO_OK;
}

}  // extern "C"
