// MTTKRP over the ALTO line (Sec. "ALTO-based Tensor Operations" and
// "Adaptive Conflict Resolution" of the paper), written for CDNA4.
//
// Work decomposition.  The ordered line is cut into L nnz-balanced tiles
// (tile l = nonzeros floor(l*M/L) .. floor((l+1)*M/L)-1, the paper's line
// segments).  Resident workgroups drain the tiles; the tiles of each XCD
// form one contiguous stretch of the line so that neighbouring tiles, which
// touch nearby factor rows, share that XCD's L2.
//
// Inside a workgroup, a "group" of LPN = R/4 (rounded up to a power of two)
// lanes owns a contiguous run of the tile's nonzeros; lane q of a group
// handles ranks 4q..4q+3 with 16-byte factor loads.  Per batch of LPN
// nonzeros each lane loads and de-linearizes one index (mask extraction,
// Fig. "alto_linear"(b)) and stages (value, output row, other coordinates)
// in LDS; then the group walks the batch in line order: it gathers the
// other modes' factor rows, forms val * Hadamard product, and merges
// consecutive updates of the same output row in registers.  When the output
// row changes, the merged row is flushed:
//   - TILE conflict resolution: into an LDS table of partial output rows
//     keyed by row (open addressing), which is added to the output once per
//     tile -- the per-partition temporary rows of the paper, keyed by row
//     instead of indexed by the mode interval, since intervals of skewed
//     tensors are far wider than LDS;
//   - RUN conflict resolution: straight to the output with global atomics.
// The output is an FP32 matrix, or an FP64 accumulation buffer that is
// rounded to FP32 once at the end (one rounding of a long sum of partials).
//
// This header holds the device code; the kernel instantiations are spread
// over several translation units (one per factor type and index width, and
// the specialised 3-mode kernels) so that they compile in parallel.
#pragma once

#include <string.h>

#include "alto_internal.h"
#include "device_util.h"
#include "mttkrp.h"

namespace alto {

namespace {

__device__ inline uint32_t row_hash(uint32_t r, int log2s) { return (r * 0x9E3779B1u) >> (32 - log2s); }

template <typename FT>
__device__ inline float4 load4(const void *base, uint64_t elem);

template <>
__device__ inline float4 load4<float>(const void *base, uint64_t elem) {
    return *(const float4 *)((const float *)base + elem);
}

__device__ inline float4 bf16x4_to_float4(uint32_t lo, uint32_t hi) {
    float4 f;
    f.x = __uint_as_float(lo << 16);
    f.y = __uint_as_float(lo & 0xFFFF0000u);
    f.z = __uint_as_float(hi << 16);
    f.w = __uint_as_float(hi & 0xFFFF0000u);
    return f;
}

template <>
__device__ inline float4 load4<uint16_t>(const void *base, uint64_t elem) {
    const uint2 u = *(const uint2 *)((const uint16_t *)base + elem);
    return bf16x4_to_float4(u.x, u.y);
}

// Factor-row gathers through a buffer resource: 32-bit byte offsets, and a
// read past the end of the factor returns zeros instead of faulting.
constexpr int kBufferFlags = 0x00020000;  // raw buffer, gfx9 family

__device__ inline __amdgpu_buffer_rsrc_t factor_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufferFlags);
}

template <typename FT>
__device__ inline float4 bload4(__amdgpu_buffer_rsrc_t r, uint32_t byte_off);

template <>
__device__ inline float4 bload4<float>(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
}

template <>
__device__ inline float4 bload4<uint16_t>(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0);
    return bf16x4_to_float4(v[0], v[1]);
}

// Gathers kept in their stored form until used: the software-pipelined
// loop issues a step's loads one step before its products, and widening
// BF16 to FP32 right after the load would make the wave wait for it there.
template <typename FT>
struct Gathered;
template <>
struct Gathered<float> {
    using T = float4;
};
template <>
struct Gathered<uint16_t> {
    using T = uint2;
};

template <typename FT>
__device__ inline typename Gathered<FT>::T bload_raw(__amdgpu_buffer_rsrc_t r, uint32_t byte_off);

template <>
__device__ inline float4 bload_raw<float>(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    return bload4<float>(r, byte_off);
}

template <>
__device__ inline uint2 bload_raw<uint16_t>(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0);
    return make_uint2(v[0], v[1]);
}

template <typename FT>
__device__ inline typename Gathered<FT>::T load_raw(const void *base, uint64_t elem);

template <>
__device__ inline float4 load_raw<float>(const void *base, uint64_t elem) {
    return load4<float>(base, elem);
}

template <>
__device__ inline uint2 load_raw<uint16_t>(const void *base, uint64_t elem) {
    return *(const uint2 *)((const uint16_t *)base + elem);
}

__device__ inline float4 widen(const float4 &v) { return v; }
__device__ inline float4 widen(const uint2 &u) { return bf16x4_to_float4(u.x, u.y); }

// Hardware id of the XCD (accelerator complex die) running this wave.
__device__ inline uint32_t xcd_id() { return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & 15u; }

// Add 4 columns of partial sums (FP32 run sums or FP64 LDS rows) to the
// output row, or to this XCD's copy of it, in FP32 or FP64.  FA: 0 reads the
// accumulation type from the arguments; the specialised kernels fix it at
// compile time (1: FP32, 2: FP64), which keeps the other form's code, and
// the registers it holds, out of them.
template <int FA = 0, typename T>
__device__ inline void global_add(const MttkrpArgs &a, uint32_t row, int r0, const T *acc) {
    uint64_t o = (uint64_t)row * a.ld + a.col0 + r0;
    if (a.copies > 1) o += (uint64_t)(xcd_id() % (uint32_t)a.copies) * a.copy_stride;
    if (FA == 2 || (FA == 0 && a.use64)) {
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (r0 + j < a.rank) unsafeAtomicAdd(a.out64 + o + j, (double)acc[j]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (r0 + j < a.rank) unsafeAtomicAdd(a.out32 + o + j, (float)acc[j]);
    }
}

// Add one column of a partial row (FP64 LDS rows or FP32 run sums) to the
// output row, or to this XCD's copy of it.  The table flushes call it with
// consecutive threads on consecutive columns of a row, so that one atomic
// instruction covers up to 16 columns (64 bytes) of a row: the L2 takes one
// request per instruction and row segment, and 4-column pieces per lane
// would cost four requests for the same 64 bytes.
template <int FA = 0, typename T>
__device__ inline void global_add1(const MttkrpArgs &a, uint32_t row, int c, T v) {
    uint64_t o = (uint64_t)row * a.ld + a.col0 + c;
    if (a.copies > 1) o += (uint64_t)(xcd_id() % (uint32_t)a.copies) * a.copy_stride;
    if (FA == 2 || (FA == 0 && a.use64)) unsafeAtomicAdd(a.out64 + o, (double)v);
    else unsafeAtomicAdd(a.out32 + o, (float)v);
}

// (slot, column) of flat element i of a table of rows with `rank` columns.
__device__ inline void split_elem(int i, int rank, int sh, int *slot, int *c) {
    *slot = sh >= 0 ? (i >> sh) : i / rank;
    *c = i - *slot * rank;
}

// Slot of `row` in the LDS table of partial rows, inserting it if absent.
// The table is bucketized: a row lives in one of the 4 slots of its bucket,
// read with a single 16-byte LDS load; an absent row takes the first empty
// slot with one compare-and-swap.  kNoSlot when the bucket is full or the
// swap lost a race: the caller then adds to the output directly.  A row may
// own two slots of its bucket (after an eviction, or two racing inserts);
// every slot is added to the output with its own key, so this only costs
// merging, never correctness.  One read and at most one swap keep the
// lookup's chain of dependent LDS round trips short.
__device__ inline uint32_t table_slot(uint32_t *tkey, uint32_t row, int log2s) {
    const uint32_t b = row_hash(row, log2s - 2) & ((1u << (log2s - 2)) - 1);
    uint32_t *bk = tkey + 4 * b;
    const uint4 k4 = *(const uint4 *)bk;
    const uint32_t kk[4] = {k4.x, k4.y, k4.z, k4.w};
#pragma unroll
    for (int j = 0; j < 4; j++)
        if (kk[j] == row) return 4 * b + j;
    int e = -1;
#pragma unroll
    for (int j = 3; j >= 0; j--)
        if (kk[j] == kEmptyRow) e = j;
    if (e >= 0) {
        const uint32_t old = atomicCAS(bk + e, kEmptyRow, row);
        if (old == kEmptyRow || old == row) return 4 * b + e;
    }
    return kNoSlot;
}

// Slot of `row` in the read-only table of a workgroup's hot rows (filled by
// hot_select), or kNoSlot: one 16-byte LDS read of the row's bucket.
__device__ inline uint32_t hot_slot(const uint32_t *tkey, uint32_t row, int log2s) {
    const uint32_t b = row_hash(row, log2s - 2);
    const uint4 k4 = *(const uint4 *)(tkey + 4 * b);
    return k4.x == row ? 4 * b : k4.y == row ? 4 * b + 1 : k4.z == row ? 4 * b + 2 : k4.w == row ? 4 * b + 3 : kNoSlot;
}

// Destination of a nonzero's update, packed in one word: kSlotBit | slot for
// an LDS slot, else the output row itself (rows are below 2^31).
constexpr uint32_t kSlotBit = 0x80000000u;

// FP32 add to 4 LDS words by compare-and-swap, the 4 swaps of a round in
// flight together.  gfx950's LDS runs ds_add_f32 about 12x slower than a
// swap loop (193 against 16 CU-cycles per wave instruction, measured with
// distinct addresses); a lost race retries with the value the swap returned.
__device__ inline void lds_add4_f32(float *t, const float *v, int n) {
    uint32_t *u = (uint32_t *)t;
    uint32_t old[4];
    bool todo[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        todo[j] = j < n;
        old[j] = todo[j] ? u[j] : 0u;
    }
    while (todo[0] || todo[1] || todo[2] || todo[3]) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (todo[j]) {
                const uint32_t want = __float_as_uint(__uint_as_float(old[j]) + v[j]);
                const uint32_t got = atomicCAS(u + j, old[j], want);
                todo[j] = got != old[j];
                old[j] = got;
            }
        }
    }
}

// Add a finished run of updates to its destination.  LDS rows are FP64:
// gfx950's LDS adds FP64 atomically about twenty times faster than FP32
// (ds_add_f64 against ds_add_f32), and the partial sums gain precision.  A
// whole-mode table whose FP64 rows would not fit (a.tw == 1) holds FP32 rows,
// twice the columns per pass, added by compare-and-swap.
template <int TM, int FA>
__device__ inline void flush_run(const MttkrpArgs &a, void *tval, uint32_t *thits, uint32_t dst, int q, int r0,
                                 const float *acc) {
    if (dst & kSlotBit) {
        const uint32_t slot = dst & ~kSlotBit;
        const int tm = TM >= 0 ? TM : a.tile_merge;
        if (tm == 2 && a.tw == 1) {
            lds_add4_f32((float *)tval + (uint64_t)slot * (a.rank + 1) + r0, acc, a.rank - r0);
            return;
        }
        double *t = (double *)tval + (uint64_t)slot * (a.rank + 1) + r0;
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (r0 + j < a.rank)
                __hip_atomic_fetch_add(t + j, (double)acc[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (q == 0 && tm == 1)
            __hip_atomic_fetch_add(thits + slot, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        global_add<FA>(a, dst, r0, acc);
    }
}

constexpr uint32_t kFlushMark = 0xFFFFFFFFu;

// ---- per-wave outbox of merged rows bound for the output
//
// A group (LPN lanes, 4 columns each) that flushes a run straight to the
// output would issue 4 atomic instructions per row, each covering 4 lanes:
// the L2 takes one request per instruction and 64-byte row segment, so a
// 16-column row costs 4 requests.  Instead the group appends the row to its
// wave's outbox in LDS, and the wave later adds whole rows with consecutive
// lanes on consecutive columns (one request per 64-byte segment).  Slots are
// assigned by a ballot over the groups that flush in the same instruction;
// the count lives in LDS (one word per wave) so that lanes that left a loop
// early and rejoin see it.  A full outbox falls back to direct atomics.
struct Outbox {
    uint32_t *rows;   // cap row indices
    float *vals;      // cap x rank columns
    uint32_t *count;  // entries in use (this wave's word)
    int cap;
};

// Outbox slots per wave for `lpn` lanes per group: two per group, so that a
// drain after every record (at most one entry per group) never overflows.
__host__ __device__ inline int outbox_cap(int lpn) { return 2 * (64 / lpn); }

__device__ inline Outbox outbox_of(uint32_t *obase, uint32_t *counts, int rank, int lpn) {
    const int cap = outbox_cap(lpn);
    const int w = threadIdx.x >> 6;
    uint32_t *p = obase + (size_t)w * cap * (rank + 1);
    return Outbox{p, (float *)(p + cap), counts + w, cap};
}

// Add every row of the outbox to the output, the wave's active lanes taking
// consecutive columns; empties the outbox.  `n` is the entry count held in
// a register (the same in every active lane); the LDS word mirrors it for
// lanes that rejoin after leaving a loop early.
template <int FA>
__device__ inline void ob_drain(const Outbox &ob, const MttkrpArgs &a, uint32_t &cnt) {
    __builtin_amdgcn_wave_barrier();
    const uint32_t n = cnt;
    if (n == 0) return;
    const uint64_t act = __activemask();
    const int me = __popcll(act & ((uint64_t(1) << (threadIdx.x & 63)) - 1));
    const int na = __popcll(act);
    const int rk = a.rank;
    const int sh = (rk & (rk - 1)) == 0 ? __ffs(rk) - 1 : -1;
    for (int i = me; i < (int)n * rk; i += na) {
        int e, c;
        split_elem(i, rk, sh, &e, &c);
        global_add1<FA>(a, ob.rows[e], c, ob.vals[e * rk + c]);
    }
    __builtin_amdgcn_wave_barrier();
    cnt = 0u;
    *ob.count = 0u;
    __builtin_amdgcn_wave_barrier();
}

// Groups with `want` set (uniform inside a group) append row `row` (lane q
// holds columns r0..r0+3 in acc) to the outbox.
template <int FA>
__device__ inline void ob_put(const Outbox &ob, const MttkrpArgs &a, bool want, uint32_t row, int q, int r0,
                              const float *acc, uint32_t &cnt) {
    const uint64_t bal = __ballot(want && q == 0);
    if (bal == 0) return;
    const int lane = threadIdx.x & 63;
    const uint32_t n = cnt;
    const int pos = (int)n + __popcll(bal & ((uint64_t(1) << (lane - q)) - 1));
    if (want) {
        if (pos < ob.cap) {
            if (q == 0) ob.rows[pos] = row;
            if (r0 < a.rank) *(float4 *)(ob.vals + (size_t)pos * a.rank + r0) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        } else {
            global_add<FA>(a, row, r0, acc);
        }
    }
    __builtin_amdgcn_wave_barrier();
    const uint32_t nn = min((uint32_t)ob.cap, n + (uint32_t)__popcll(bal));
    cnt = nn;
    *ob.count = nn;
    __builtin_amdgcn_wave_barrier();
}

// Coordinate k of the other modes from a staged record held as two uint4.
__device__ inline uint32_t rec_coord(const uint4 &h, const uint4 &h2, int k) {
    return k == 0 ? h.z : k == 1 ? h.w : k == 2 ? h2.x : k == 3 ? h2.y : k == 4 ? h2.z : h2.w;
}

// End of a tile of the workgroup's tiles (`last`: its final one; `ord`: how
// many it processed before this one): the LDS table's rows go to the output
// -- for a whole-mode table (TM 2) once, after the final tile; for a hashed
// table (TM 1) every tile, except rows merged many times (high reuse), which
// stay for the next tile.  Everything is flushed every kKeepTiles tiles and
// after the final one.
template <int FA>
__device__ inline void tile_end(const MttkrpArgs &a, int TM, int TW, int S, int TS, uint32_t *tkey, uint32_t *thits,
                                void *tval, uint32_t &nkeep, bool last, uint64_t ord) {
    const int tid = threadIdx.x;
    double *tv64 = (double *)tval;
    float *tv32 = (float *)tval;
    // one column per thread (see global_add1); sh: log2(rank), or -1
    const int rk = a.rank;
    const int sh = (rk & (rk - 1)) == 0 ? __ffs(rk) - 1 : -1;
    if (TM == 2 && last) {
        // ---- end of the stretch: every row of the mode held in LDS is
        // added to the output once
        __syncthreads();
        for (int i = tid; i < S * rk; i += blockDim.x) {
            int row, c;
            split_elem(i, rk, sh, &row, &c);
            if (TW == 2) {
                const double v = tv64[(size_t)row * TS + c];
                if (v != 0.0) global_add1<FA>(a, (uint32_t)row, c, v);
            } else {
                const float v = tv32[(size_t)row * TS + c];
                if (v != 0.f) global_add1<FA>(a, (uint32_t)row, c, v);
            }
        }
        __syncthreads();
    } else if (TM == 3 && last) {
        // ---- end of the stretch: the hot rows' partial sums go to the output
        __syncthreads();
        for (int i = tid; i < S * rk; i += blockDim.x) {
            int slot, c;
            split_elem(i, rk, sh, &slot, &c);
            const uint32_t row = tkey[slot];
            if (row == kEmptyRow) continue;
            const double v = tv64[(size_t)slot * TS + c];
            if (v != 0.0) global_add1<FA>(a, row, c, v);
        }
        __syncthreads();
    } else if (TM == 1) {
        __syncthreads();
        const bool flush_all = last || ((ord + 1) % kKeepTiles == 0);
        if (tid == 0) nkeep = 0;
        __syncthreads();
        for (int i = tid; i < S; i += blockDim.x) {
            if (tkey[i] == kEmptyRow) continue;
            bool keep = false;
            if (!flush_all && thits[i] >= kHotHits) keep = atomicAdd(&nkeep, 1u) < (uint32_t)(S / 4);
            thits[i] = keep ? 0u : kFlushMark;
        }
        __syncthreads();
        for (int i = tid; i < S * rk; i += blockDim.x) {
            int slot, c;
            split_elem(i, rk, sh, &slot, &c);
            if (thits[slot] == kFlushMark) {
                double *tv = tv64 + (size_t)slot * TS + c;
                global_add1<FA>(a, tkey[slot], c, *tv);
                *tv = 0.0;
            }
        }
        __syncthreads();
        for (int i = tid; i < S; i += blockDim.x) {
            if (thits[i] == kFlushMark) {
                tkey[i] = kEmptyRow;
                thits[i] = 0;
            }
        }
        __syncthreads();
    }
}

// Compress one 64-bit index word with masks read from LDS (every lane reads
// the same address: a broadcast).
__device__ inline uint64_t compress_lds(uint64_t x, const uint64_t *m) {
    x &= m[0];
#pragma unroll
    for (int i = 0; i < 6; i++) {
        const uint64_t t = x & m[1 + i];
        x = (x ^ t) | (t >> (1u << i));
    }
    return x;
}

// Tiles [t0, t1) of one tensor's line, processed by one workgroup (the
// plain, unpipelined loop without outboxes: tensors of 6-8 modes).  The LDS
// table is initialized here and fully flushed by the last tile.  TMC: the
// conflict-resolution mode fixed at compile time (-1: read from the
// arguments).
template <int LPN, typename FT, int WORDS, int MAXO, int TMC>
__device__ inline void mttkrp_stretch(const MttkrpArgs &a, uint32_t *smem, uint32_t &nkeep, uint64_t t0, uint64_t t1) {
    const int TM = TMC >= 0 ? TMC : a.tile_merge;
    // nonzeros gathered together per group
    constexpr int SB = MAXO == 2 ? (LPN < 4 ? LPN : 4) : (LPN < 2 ? LPN : 2);
    // table rows: hashed slots (tile merge) or every row of the mode (direct).
    // Rows are rank + 1 doubles apart: the odd stride spreads the rows the
    // groups of a wave update at once over all LDS banks.
    const int S = TM == 1 ? (1 << a.slots_log2) : (TM == 2 ? (int)a.dim_out : 0);
    const int SK = TM == 1 ? S : 0;  // key / hit arrays
    const int TS = a.rank + 1;
    uint32_t *tkey = smem;
    uint32_t *thits = smem + SK;
    const int TW = TM == 2 ? a.tw : 2;             // words per table element
    void *tval = (void *)(smem + 2 * SK);          // 2 * SK is even: 8-byte aligned
    uint32_t *stage = smem + ((2 * SK + (size_t)TW * S * TS + 3) & ~(size_t)3);
    const int REC = a.rec;  // [val, destination, other coordinates...], multiple of 4
    const int tid = threadIdx.x;
    const int q = tid & (LPN - 1);
    const int grp = tid / LPN;
    const int ngrp = blockDim.x / LPN;
    uint32_t *gst = stage + grp * LPN * REC;
    const int r0 = 4 * q;
    const bool ract = r0 < a.rank;
    const int nother = a.nmodes - 1;

    if (TM) {
        for (int i = tid; i < SK; i += blockDim.x) {
            tkey[i] = kEmptyRow;
            thits[i] = 0;
        }
        for (int i = tid; i < TW * S * TS; i += blockDim.x) smem[2 * SK + i] = 0u;
        __syncthreads();
    }

    for (uint64_t t = t0; t < t1; t++) {
        const uint64_t ts = t * a.tq + (t * a.tr) / a.ntiles;
        const uint64_t te = (t + 1) * a.tq + ((t + 1) * a.tr) / a.ntiles;
        const uint64_t per = (te - ts + ngrp - 1) / ngrp;
        uint64_t ga = ts + (uint64_t)grp * per;
        if (ga > te) ga = te;
        const uint64_t gb = (ga + per < te) ? ga + per : te;

        uint32_t cur = kEmptyRow;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};

        // index and value of this lane's next nonzero, loaded one batch ahead
        uint64_t nlo = 0, nhi = 0;
        float nval = 0.f;
        if (ga + q < gb) {
            nlo = a.keys[(ga + q) * WORDS];
            if (WORDS == 2) nhi = a.keys[(ga + q) * WORDS + 1];
            nval = a.vals[ga + q];
        }
        for (uint64_t base = ga; base < gb; base += LPN) {
            const uint64_t x = base + q;
            const uint64_t lo = nlo, hi = nhi;
            const float val = nval;
            if (x + LPN < gb) {
                nlo = a.keys[(x + LPN) * WORDS];
                if (WORDS == 2) nhi = a.keys[(x + LPN) * WORDS + 1];
                nval = a.vals[x + LPN];
            }
            // ---- one nonzero per lane: de-linearize, find its LDS slot, stage
            uint32_t *rec = gst + q * REC;
            if (x < gb) {
                uint32_t c3[3] = {0u, 0u, 0u};
                uint32_t row;
                if (MAXO == 2 && WORDS == 1) {
#pragma unroll
                    for (int m = 0; m < 3; m++)
                        if (m < a.nmodes) c3[m] = extract_mode<1>(a.lp.mode[m], lo, hi);
                    row = a.mode == 0 ? c3[0] : (a.mode == 1 ? c3[1] : c3[2]);
                } else {
                    row = extract_mode<WORDS>(a.lp.mode[a.mode], lo, hi);
                }
                // indices decode from valid coordinates; the checks below only
                // keep a corrupted index from reaching memory
                const bool row_ok = row < a.dim_out;
                uint32_t dst = kEmptyRow;
                if (row_ok) {
                    dst = row;
                    if (TM == 1) {
                        const uint32_t slot = table_slot(tkey, row, a.slots_log2);
                        if (slot != kNoSlot) dst = kSlotBit | slot;
                    } else if (TM == 2) {
                        dst = kSlotBit | row;
                    }
                }
                if (MAXO == 2 && WORDS == 1) {
                    // up to 3 modes: the masks stay in scalar registers, and
                    // the record is one 16-byte LDS store
                    const uint32_t o0 = a.mode == 0 ? c3[1] : c3[0];
                    const uint32_t o1 = a.mode == 2 ? c3[1] : c3[2];
                    *(uint4 *)rec = make_uint4(row_ok ? __float_as_uint(val) : 0u, dst, o0, o1);
                } else {
                    rec[0] = row_ok ? __float_as_uint(val) : 0u;
                    rec[1] = dst;
                    // modes in a rolled loop: each mode's masks are fetched
                    // into scalar registers when needed instead of all at once
                    int k = 2;
#pragma unroll 1
                    for (int m = 0; m < a.nmodes; m++) {
                        if (m != a.mode) {
                            rec[k] = extract_mode<WORDS>(a.lp.mode[m], lo, hi);
                            k++;
                        }
                    }
                }
            } else if (MAXO == 2 && WORDS == 1) {
                *(uint4 *)rec = make_uint4(0u, kEmptyRow, 0u, 0u);
            } else {
                rec[0] = 0u;
                rec[1] = kEmptyRow;
                for (int k = 2; k < 2 + nother; k++) rec[k] = 0u;
            }
            __builtin_amdgcn_wave_barrier();
            const int cnt = (int)((gb - base) < (uint64_t)LPN ? (gb - base) : (uint64_t)LPN);

            // ---- walk the batch in line order
#pragma unroll
            for (int sb = 0; sb < LPN; sb += SB) {
                float p[SB][4];
                uint4 head[SB], head2[SB];
#pragma unroll
                for (int s = 0; s < SB; s++) {
                    head[s] = *(const uint4 *)(gst + (sb + s) * REC);
                    head2[s] = (MAXO > 2 && nother > 2) ? *(const uint4 *)(gst + (sb + s) * REC + 4)
                                                        : make_uint4(0, 0, 0, 0);
                    const float v = __uint_as_float(head[s].x);
                    p[s][0] = v;
                    p[s][1] = v;
                    p[s][2] = v;
                    p[s][3] = v;
                }
                if (MAXO <= 4) {
                    // every gather of the batch is issued before the first
                    // product is formed
                    float4 g[MAXO][SB];
#pragma unroll
                    for (int k = 0; k < MAXO; k++) {
                        if (k < nother) {
                            if (a.buf32) {
                                const __amdgpu_buffer_rsrc_t rs = factor_rsrc(a.fac_other[k], a.fac_bytes[k]);
#pragma unroll
                                for (int s = 0; s < SB; s++) {
                                    const uint32_t idx = rec_coord(head[s], head2[s], k);
                                    g[k][s] = bload4<FT>(rs, (idx * a.ld + a.col0 + (uint32_t)r0) * (uint32_t)sizeof(FT));
                                }
                            } else {
                                const void *f = a.fac_other[k];
#pragma unroll
                                for (int s = 0; s < SB; s++) {
                                    const uint32_t idx = min(rec_coord(head[s], head2[s], k), a.last_other[k]);
                                    g[k][s] = ract ? load4<FT>(f, (uint64_t)idx * a.ld + a.col0 + r0)
                                                   : make_float4(0.f, 0.f, 0.f, 0.f);
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < MAXO; k++) {
                        if (k < nother) {
#pragma unroll
                            for (int s = 0; s < SB; s++) {
                                p[s][0] *= g[k][s].x;
                                p[s][1] *= g[k][s].y;
                                p[s][2] *= g[k][s].z;
                                p[s][3] *= g[k][s].w;
                            }
                        }
                    }
                } else {
                    for (int k = 0; k < nother; k++) {
                        const void *f = a.fac_other[k];
#pragma unroll
                        for (int s = 0; s < SB; s++) {
                            const uint32_t idx = min(gst[(sb + s) * REC + 2 + k], a.last_other[k]);
                            const float4 g = ract ? load4<FT>(f, (uint64_t)idx * a.ld + a.col0 + r0)
                                                  : make_float4(0.f, 0.f, 0.f, 0.f);
                            p[s][0] *= g.x;
                            p[s][1] *= g.y;
                            p[s][2] *= g.z;
                            p[s][3] *= g.w;
                        }
                    }
                }
#pragma unroll
                for (int s = 0; s < SB; s++) {
                    if (sb + s < cnt) {
                        const uint32_t dst = head[s].y;
                        if (dst == cur) {
#pragma unroll
                            for (int j = 0; j < 4; j++) acc[j] += p[s][j];
                        } else {
                            if (cur != kEmptyRow) flush_run<TMC, false>(a, tval, thits, cur, q, r0, acc);
                            cur = dst;
#pragma unroll
                            for (int j = 0; j < 4; j++) acc[j] = p[s][j];
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (cur != kEmptyRow) flush_run<TMC, false>(a, tval, thits, cur, q, r0, acc);

        tile_end<false>(a, TM, TW, S, TS, tkey, thits, tval, nkeep, t + 1 == t1, t - t0);
    }
}

// Extraction masks of every mode in LDS, per mode kMaskStride words: for
// each index word the AND mask and the 6 move masks, then (two-word
// indices) the number of the mode's bits held in word 0.  All lanes read the
// same address, so every read is a broadcast.
constexpr int kMaskStride = 15;
constexpr int kMaskWords = ALTO_MAX_MODES * kMaskStride;

// Fill `lm` from the plan (all threads of the block call it; ends with a
// barrier).
__device__ inline void load_masks(const LinePlan &lp, int nmodes, uint64_t *lm) {
    for (int i = threadIdx.x; i < nmodes * kMaskStride; i += blockDim.x) {
        const int m = i / kMaskStride, k = i - m * kMaskStride;
        const ModeMasks &mm = lp.mode[m];
        uint64_t v;
        if (k < 14) {
            const WordMasks &w = mm.w[k / 7];
            v = k % 7 == 0 ? w.mask : w.mv[k % 7 - 1];
        } else {
            v = (uint64_t)mm.lo_bits;
        }
        lm[i] = v;
    }
    __syncthreads();
}

// Coordinates of a 3-mode, one-word index whose modes have at most 21 bits
// each, from a table of 16 nibble positions x 16 values in LDS: entry (c, v)
// holds the bits of nibble c = v deposited into three 21-bit fields (mode m
// at bit 21 m).  One LDS read and an OR per nibble replace
// the three mask compressions (each six 64-bit steps with LDS masks).
constexpr int kLutNibbles = 16;

__device__ inline void build_nibble_lut(const uint64_t *lm, uint64_t *lut) {
    for (int t = threadIdx.x; t < kLutNibbles * 16; t += blockDim.x) {
        const int c = t >> 4, v = t & 15;
        uint64_t e = 0;
        for (int b = 0; b < 4; b++) {
            if (!((v >> b) & 1)) continue;
            const int p = 4 * c + b;
            for (int m = 0; m < 3; m++) {
                const uint64_t mask = lm[m * kMaskStride];  // word-0 mask of mode m
                if ((mask >> p) & 1) e |= uint64_t(1) << (21 * m + __popcll(mask & ((uint64_t(1) << p) - 1)));
            }
        }
        lut[t] = e;
    }
    __syncthreads();
}

// Used by the specialised kernel at up to 4 lanes per nonzero (rank <= 16),
// where decoding is a large share of each lane's work: c2 (R=16) MTTKRP
// calls 2.08 / 2.06 / 2.18 -> 2.02 / 1.98 / 2.12 ms.  At 16 lanes (R=64)
// one decode serves 16 lanes' gathers and products, and the table's LDS
// reads measured slower (8.4 -> 8.6 ms and 8.9 -> 9.2 ms on modes 1 and 2).
template <bool FAST, int WORDS, int LPN>
constexpr bool kUseLut = FAST && WORDS == 1 && LPN <= 4;

__device__ inline uint64_t lut_decode(const uint64_t *lut, uint64_t x) {
    uint64_t acc = 0;
#pragma unroll
    for (int c = 0; c < kLutNibbles; c++) acc |= lut[c * 16 + (int)((x >> (4 * c)) & 15u)];
    return acc;
}

// Coordinate of mode m from an index (lo, hi) with the masks in LDS.
template <int WORDS>
__device__ inline uint32_t extract_lds(const uint64_t *lm, int m, uint64_t lo, uint64_t hi) {
    const uint64_t *mm = lm + m * kMaskStride;
    uint64_t c = compress_lds(lo, mm);
    if (WORDS == 2) c |= compress_lds(hi, mm + 7) << (uint32_t)mm[14];
    return (uint32_t)c;
}

// Hot rows of one workgroup's line stretch [z0, z1) (HOT conflict
// resolution).  Skewed tensors send most updates of a stretch to a few
// hundred rows, but the rows differ from stretch to stretch, so each
// workgroup picks its own: it counts the output rows of an evenly strided
// sample of its nonzeros in an LDS hash table (linear probing), keeps the
// at most 3S/4 rows seen most often (at least twice), and places them in
// the bucketed table tkey of S slots, where they stay for the whole stretch
// (a row whose bucket is full stays cold).  Every other row's updates merge
// in registers and go to the output directly.  LDS use: the sample table
// overlays the partial-row area `work` (work_words words, cleared at the
// end for the rows), the selected rows go to `list` (S words), and `hist`
// (>= 260 words of the record staging) holds a histogram of the counts.
constexpr uint32_t kHotMin = 2;           // sample hits that make a row a candidate
constexpr int kHotSampleMax = 12288;      // samples per stretch
constexpr int kHotProbe = 32;             // sample-table probes before a sample is dropped

template <int WORDS>
__device__ void hot_select(const MttkrpArgs &a, const uint64_t *lmask, uint64_t z0, uint64_t z1, uint32_t *tkey,
                           uint32_t *list, uint32_t *work, size_t work_words, uint32_t *hist, int S) {
    const int tid = threadIdx.x, bd = blockDim.x;
    // sample table: ST keys then ST counts
    uint32_t log2t = 4;
    while (log2t < 15 && ((size_t)2 << (log2t + 1)) <= work_words) log2t++;
    const uint32_t ST = 1u << log2t;
    uint32_t *skey = work, *scnt = work + ST;
    for (uint32_t i = tid; i < ST; i += bd) {
        skey[i] = kEmptyRow;
        scnt[i] = 0u;
    }
    for (int i = tid; i < 260; i += bd) hist[i] = 0u;
    __syncthreads();
    const uint64_t n = z1 > z0 ? z1 - z0 : 0;
    const uint64_t cap = (uint64_t)min((uint32_t)kHotSampleMax, ST / 4 * 3);
    const uint64_t nsamp = n < cap ? n : cap;
    const uint64_t stride = nsamp ? (n + nsamp - 1) / nsamp : 1;
    for (uint64_t j = tid; j < nsamp; j += bd) {
        const uint64_t x = z0 + j * stride;
        if (x >= z1) break;
        const uint64_t lo = a.keys[x * WORDS];
        const uint64_t hi = WORDS == 2 ? a.keys[x * WORDS + 1] : 0;
        const uint32_t row = extract_lds<WORDS>(lmask, a.mode, lo, hi);
        if (row >= a.dim_out) continue;
        uint32_t h = row_hash(row, (int)log2t);
        for (int p = 0; p < kHotProbe; p++) {
            const uint32_t k = skey[h];
            if (k == kEmptyRow) {
                const uint32_t old = atomicCAS(skey + h, kEmptyRow, row);
                if (old == kEmptyRow || old == row) {
                    atomicAdd(scnt + h, 1u);
                    break;
                }
            } else if (k == row) {
                atomicAdd(scnt + h, 1u);
                break;
            }
            h = (h + 1) & (ST - 1);
        }
    }
    __syncthreads();
    // histogram of the counts (255 = 255 or more), threshold for the top kmax
    for (uint32_t i = tid; i < ST; i += bd) {
        const uint32_t c = scnt[i];
        if (c >= kHotMin) atomicAdd(hist + min(c, 255u), 1u);
    }
    __syncthreads();
    const uint32_t kmax = (uint32_t)S / 4 * 3;
    if (tid == 0) {
        uint32_t above = 0, cstar = kHotMin, take = hist[kHotMin];
        for (uint32_t c = 255; c >= kHotMin; c--) {
            if (above + hist[c] >= kmax) {
                cstar = c;
                take = kmax - above;
                break;
            }
            above += hist[c];
        }
        hist[256] = cstar;
        hist[257] = take;
        hist[258] = 0u;  // selected
        hist[259] = 0u;  // taken at the threshold
    }
    __syncthreads();
    const uint32_t cstar = hist[256], take = hist[257];
    for (uint32_t i = tid; i < ST; i += bd) {
        const uint32_t c = min(scnt[i], 255u);
        if (c < kHotMin || c < cstar) continue;
        if (c == cstar && atomicAdd(hist + 259, 1u) >= take) continue;
        list[atomicAdd(hist + 258, 1u)] = skey[i];
    }
    __syncthreads();
    const uint32_t nsel = hist[258];
    const int log2s = a.slots_log2;
    for (int i = tid; i < S; i += bd) tkey[i] = kEmptyRow;
    for (size_t i = tid; i < work_words; i += bd) work[i] = 0u;
    __syncthreads();
    for (uint32_t i = tid; i < nsel; i += bd) {
        const uint32_t row = list[i];
        uint32_t *bk = tkey + 4 * row_hash(row, log2s - 2);
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (atomicCAS(bk + j, kEmptyRow, row) == kEmptyRow) break;
    }
    __syncthreads();
}

// Software-pipelined stretch for tensors of up to 5 modes (MAXO = most
// other modes: 2 or 4): the next batch is de-linearized, looked up and
// staged, and the gathers of its next step issued, before the products and
// merges of the current step -- so the gathers' latency overlaps this
// step's LDS work.  A group stages a batch in one buffer of LPN records of
// RW words (value, destination, the other coordinates): every record of the
// previous batch is already in registers when the next batch overwrites it
// (a wave's LDS operations execute in order).  The two register sets of a
// step (X and Y) alternate by hand, so nothing is copied.  FAST: exactly 3
// modes, one-word index and 32-bit buffer gathers (the specialised kernel);
// FA: the accumulation type, fixed at compile time there (see global_add).
//
// OP selects what is accumulated per nonzero x (coordinates i, value v):
//   kOpMttkrp: v * krp, krp = Hadamard product of the other factors' rows;
//   kOpPhi:    v / max(B(i_mode, :) . krp, eps) * krp -- the CP-APR model
//              update Phi (Algorithm "alg:cp-apr-mu", Phi line; Algorithm
//              "fig:subproblem_algo" with krp computed on the fly, ALTO-OTF);
//   kOpPhiPre: the same with krp read as row x of a precomputed Pi (ALTO-PRE).
// For the Phi forms the group's LPN lanes hold the whole rank (no rank
// tiles): each lane forms its 4 columns of B(i_mode, :) . krp and a
// butterfly of lane shuffles inside the group completes the dot product.
// Their records are 8 words: the output row is kept in the last word (the
// destination word may name an LDS slot instead), and kOpPhiPre keeps the
// nonzero's position in the first coordinate word.
constexpr int kOpMttkrp = 0, kOpPhi = 1, kOpPhiPre = 2;

template <int LPN, typename FT, int WORDS, int MAXO, int TMC, bool FAST, int OP = kOpMttkrp, int FA = 0>
__device__ inline void mttkrp_stretch_pipe(const MttkrpArgs &a, uint32_t *smem, uint32_t &nkeep,
                                           const uint64_t *lmask, uint64_t t0, uint64_t t1,
                                           const uint64_t *lut = nullptr, uint64_t tstep = 1) {
    static_assert(MAXO == 2 || MAXO == 4, "pipelined stretch: up to 5 modes");
    static_assert(OP == kOpMttkrp || (MAXO == 4 && !FAST), "Phi forms use 8-word records");
    const int TM = TMC >= 0 ? TMC : a.tile_merge;
    using GT = typename Gathered<FT>::T;
    constexpr int SB = MAXO == 2 ? (LPN < 4 ? LPN : 4) : (LPN < 2 ? LPN : 2);  // records per step
    constexpr int NS = LPN / SB;                                               // steps per batch
    constexpr int RW = MAXO == 2 ? 4 : 8;                                      // record words
    const int nmodes = FAST ? 3 : a.nmodes;
    // the rows multiplied per nonzero: the other modes' (or the one Pi row)
    const int nother = OP == kOpPhiPre ? 1 : nmodes - 1;
    const int S = (TM == 1 || TM == 3) ? (1 << a.slots_log2) : (TM == 2 ? (int)a.dim_out : 0);
    const int SK = (TM == 1 || TM == 3) ? S : 0;
    const int TS = a.rank + 1;
    uint32_t *tkey = smem;
    uint32_t *thits = smem + SK;
    const int TW = a.tw;
    void *tval = (void *)(smem + 2 * SK);
    uint32_t *stage = smem + ((2 * SK + (size_t)TW * S * TS + 3) & ~(size_t)3);
    const int tid = threadIdx.x;
    const int q = tid & (LPN - 1);
    const int grp = tid / LPN;
    const int ngrp = blockDim.x / LPN;
    uint32_t *gbuf = stage + grp * LPN * RW;
    const int r0 = 4 * q;
    const bool ract = r0 < a.rank;
    const bool buf32 = FAST || a.buf32;
    // the outbox follows the record staging (none for the whole-mode table,
    // whose rows are all in LDS)
    __shared__ uint32_t ob_counts[16];
    if ((tid & 63) == 0) ob_counts[tid >> 6] = 0u;
    const Outbox ob = outbox_of(stage + (size_t)ngrp * LPN * RW, ob_counts, a.rank, LPN);
    uint32_t obn = 0u;  // the wave's outbox entries (see ob_drain)
    constexpr int kGroupsPerWave = 64 / LPN;
    __amdgpu_buffer_rsrc_t rs[MAXO];
#pragma unroll
    for (int k = 0; k < MAXO; k++)
        if (k < nother) rs[k] = factor_rsrc(a.fac_other[k], a.fac_bytes[k]);
    const uint32_t ldb = a.ld * (uint32_t)sizeof(FT);
    const uint32_t colb = (a.col0 + (uint32_t)r0) * (uint32_t)sizeof(FT);
    const int mode = a.mode;

    if (TM == 3) {
        const uint64_t z0 = t0 * a.tq + (t0 * a.tr) / a.ntiles;
        const uint64_t z1 = t1 * a.tq + (t1 * a.tr) / a.ntiles;
        hot_select<WORDS>(a, lmask, z0, z1, tkey, thits, (uint32_t *)tval, (size_t)TW * S * TS, stage, S);
    } else if (TM) {
        for (int i = tid; i < SK; i += blockDim.x) {
            tkey[i] = kEmptyRow;
            thits[i] = 0;
        }
        for (int i = tid; i < TW * S * TS; i += blockDim.x) smem[2 * SK + i] = 0u;
        __syncthreads();
    }

    for (uint64_t t = t0; t < t1; t += tstep) {
        const uint64_t ts = t * a.tq + (t * a.tr) / a.ntiles;
        const uint64_t te = (t + 1) * a.tq + ((t + 1) * a.tr) / a.ntiles;
        const uint64_t per = (te - ts + ngrp - 1) / ngrp;
        uint64_t ga = ts + (uint64_t)grp * per;
        if (ga > te) ga = te;
        const uint64_t gb = (ga + per < te) ? ga + per : te;
        const uint64_t nsteps = (gb - ga + LPN - 1) / LPN * NS;

        uint32_t cur = kEmptyRow;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        // index and value of this lane's nonzero in the next batch
        uint64_t nlo = 0, nhi = 0;
        float nval = 0.f;
        if (ga + q < gb) {
            nlo = a.keys[(ga + q) * WORDS];
            if (WORDS == 2) nhi = a.keys[(ga + q) * WORDS + 1];
            nval = a.vals[ga + q];
        }

        // batch b: one nonzero per lane de-linearized, looked up, staged
        auto decode = [&](uint64_t b) {
            const uint64_t x = ga + b * LPN + q;
            const uint64_t lo = nlo, hi = nhi;
            const float val = nval;
            if (x + LPN < gb) {
                nlo = a.keys[(x + LPN) * WORDS];
                if (WORDS == 2) nhi = a.keys[(x + LPN) * WORDS + 1];
                nval = a.vals[x + LPN];
            }
            uint32_t r[RW];
#pragma unroll
            for (int k = 0; k < RW; k++) r[k] = 0u;
            r[1] = kEmptyRow;
            if (x < gb) {
                uint32_t c[MAXO + 1];
                if (kUseLut<FAST, WORDS, LPN> && a.lut) {
                    const uint64_t e = lut_decode(lut, lo);
                    c[0] = (uint32_t)(e & 0x1FFFFFu);
                    c[1] = (uint32_t)((e >> 21) & 0x1FFFFFu);
                    c[2] = (uint32_t)(e >> 42);
                } else {
#pragma unroll
                    for (int m = 0; m <= MAXO; m++) c[m] = m < nmodes ? extract_lds<WORDS>(lmask, m, lo, hi) : 0u;
                }
                uint32_t row = c[0];
#pragma unroll
                for (int m = 1; m <= MAXO; m++)
                    if (m == mode) row = c[m];
                // indices decode from valid coordinates; the check only keeps
                // a corrupted index from reaching memory
                if (row < a.dim_out) {
                    uint32_t dst = row;
                    if (TM == 1) {
                        const uint32_t slot = table_slot(tkey, row, a.slots_log2);
                        if (slot != kNoSlot) dst = kSlotBit | slot;
                    } else if (TM == 2) {
                        dst = kSlotBit | row;
                    } else if (TM == 3) {
                        const uint32_t slot = hot_slot(tkey, row, a.slots_log2);
                        if (slot != kNoSlot) dst = kSlotBit | slot;
                    }
                    r[0] = __float_as_uint(val);
                    r[1] = dst;
#pragma unroll
                    for (int k = 0; k < MAXO; k++) r[2 + k] = k < mode ? c[k] : c[k + 1];
                    if (OP == kOpPhiPre) r[2] = (uint32_t)x;
                    if (OP != kOpMttkrp) r[RW - 1] = row;
                }
            }
            uint32_t *rec = gbuf + q * RW;
            *(uint4 *)rec = make_uint4(r[0], r[1], r[2], r[3]);
            if (RW == 8) *(uint4 *)(rec + 4) = make_uint4(r[4], r[5], r[6], r[7]);
        };
        // step k: its records' heads, and the gathers of the other modes
        // (Phi forms: and of B's row of the output mode)
        auto issue = [&](uint64_t k, GT (&g)[MAXO][SB], uint32_t (&dv)[SB], float (&vv)[SB],
                         float4 (&gB)[SB]) {
            if (k % NS == 0) {
                decode(k / NS);
                __builtin_amdgcn_wave_barrier();
            }
            const uint32_t *buf = gbuf + (k % NS) * SB * RW;
#pragma unroll
            for (int s = 0; s < SB; s++) {
                const uint4 h = *(const uint4 *)(buf + s * RW);
                const uint4 h2 = RW == 8 ? *(const uint4 *)(buf + s * RW + 4) : make_uint4(0u, 0u, 0u, 0u);
                dv[s] = h.y;
                vv[s] = __uint_as_float(h.x);
                const uint32_t idx[4] = {h.z, h.w, h2.x, h2.y};
                if constexpr (OP != kOpMttkrp) {
                    const bool live = ract && h.y != kEmptyRow;
                    gB[s] = live ? *(const float4 *)(a.phi_B + (uint64_t)h2.w * a.ld + r0)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
                }
                if constexpr (OP == kOpPhiPre) {
                    const bool live = ract && h.y != kEmptyRow;
                    g[0][s] = live ? *(const float4 *)(a.phi_pi + (uint64_t)h.z * a.ld + r0)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
                    continue;
                }
#pragma unroll
                for (int k2 = 0; k2 < MAXO; k2++) {
                    if (k2 < nother) {
                        if (buf32) {
                            g[k2][s] = bload_raw<FT>(rs[k2], idx[k2] * ldb + colb);
                        } else {
                            const uint32_t ii = min(idx[k2], a.last_other[k2]);
                            g[k2][s] = ract ? load_raw<FT>(a.fac_other[k2], (uint64_t)ii * a.ld + a.col0 + r0)
                                            : GT{};
                        }
                    }
                }
            }
        };
        // products of a step, merged into runs of equal destinations; a
        // finished run goes to its LDS slot, or to the wave's outbox
        auto consume = [&](const GT (&g)[MAXO][SB], const uint32_t (&dv)[SB], const float (&vv)[SB],
                           const float4 (&gB)[SB]) {
#pragma unroll
            for (int s = 0; s < SB; s++) {
                const bool live = dv[s] != kEmptyRow;
                const float v0 = OP == kOpMttkrp ? vv[s] : 1.f;
                float p[4] = {v0, v0, v0, v0};
#pragma unroll
                for (int k2 = 0; k2 < MAXO; k2++) {
                    if (k2 < nother) {
                        const float4 gv = widen(g[k2][s]);
                        p[0] *= gv.x;
                        p[1] *= gv.y;
                        p[2] *= gv.z;
                        p[3] *= gv.w;
                    }
                }
                if constexpr (OP != kOpMttkrp) {
                    // the model at this nonzero, B(i_mode, :) . krp, over the group
                    float d = gB[s].x * p[0] + gB[s].y * p[1] + gB[s].z * p[2] + gB[s].w * p[3];
#pragma unroll
                    for (int o = 1; o < LPN; o <<= 1) d += __shfl_xor(d, o, 64);
                    const float sc = vv[s] / fmaxf(d, a.phi_eps);
#pragma unroll
                    for (int j = 0; j < 4; j++) p[j] *= sc;
                }
                const bool same = live && dv[s] == cur;
                const bool fl = live && !same && cur != kEmptyRow;
                ob_put<FA>(ob, a, fl && !(cur & kSlotBit), cur, q, r0, acc, obn);
                if (fl && (cur & kSlotBit)) flush_run<TMC, FA>(a, tval, thits, cur, q, r0, acc);
                if (same) {
#pragma unroll
                    for (int j = 0; j < 4; j++) acc[j] += p[j];
                } else if (live) {
                    cur = dv[s];
#pragma unroll
                    for (int j = 0; j < 4; j++) acc[j] = p[j];
                }
                if (obn > (uint32_t)(ob.cap - kGroupsPerWave)) ob_drain<FA>(ob, a, obn);
            }
        };

        GT xg[MAXO][SB], yg[MAXO][SB];
        float4 xb[SB], yb[SB];
        uint32_t xd[SB], yd[SB];
        float xv[SB], yv[SB];
        if (nsteps > 0) issue(0, xg, xd, xv, xb);
        for (uint64_t k = 0; k < nsteps; k += 2) {
            if (k + 1 < nsteps) issue(k + 1, yg, yd, yv, yb);
            consume(xg, xd, xv, xb);
            if (k + 1 >= nsteps) break;
            if (k + 2 < nsteps) issue(k + 2, xg, xd, xv, xb);
            consume(yg, yd, yv, yb);
        }
        {
            // groups that left the step loop early rejoin here: the LDS word
            // holds the count the last active lanes left
            __builtin_amdgcn_wave_barrier();
            obn = *(volatile uint32_t *)ob.count;
            const bool fl = cur != kEmptyRow;
            ob_put<FA>(ob, a, fl && !(cur & kSlotBit), cur, q, r0, acc, obn);
            if (fl && (cur & kSlotBit)) flush_run<TMC, FA>(a, tval, thits, cur, q, r0, acc);
        }
        ob_drain<FA>(ob, a, obn);
        __builtin_amdgcn_wave_barrier();
        tile_end<FA>(a, TM, TW, S, TS, tkey, thits, tval, nkeep, t + tstep >= t1, (t - t0) / tstep);
    }
}

// Balanced stretch [g0, g1) of `total` tiles for this workgroup.  The
// stretches of the workgroups that share an XCD (block id mod 8) are
// neighbours on the line, so the factor rows they touch share its L2.
__device__ inline void stretch_of(uint64_t total, int xcd_map, uint64_t *g0, uint64_t *g1) {
    const uint32_t G = gridDim.x;
    const uint32_t rr = xcd_map ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
    *g0 = (total * rr) / G;
    *g1 = (total * (rr + 1)) / G;
}

// Kernel variants: MAXO = most other modes handled with fully unrolled
// gathers (2: up to 3-mode tensors, 4: up to 5 modes); 7: any order, rolled.
template <int LPN, typename FT, int WORDS, int MAXO, int TMC, bool FAST, bool F64 = false>
__global__ __launch_bounds__(512) void k_mttkrp(const MttkrpArgs a) {
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ uint32_t nkeep;
    __shared__ uint64_t lmask[(FAST || MAXO <= 4) ? kMaskWords : 1];
    __shared__ uint64_t lut[kUseLut<FAST, WORDS, LPN> ? kLutNibbles * 16 : 1];
    uint64_t t0, t1;
    stretch_of(a.ntiles, a.xcd_map, &t0, &t1);
    // the pipelined loop (with the per-wave outboxes) for up to 5 modes; the
    // plain loop for 6-8 modes
    if constexpr (FAST || MAXO <= 4) {
        uint64_t tstep = 1;
        if (a.xcd_map && a.interleave) {
            // the XCD's tiles (the same contiguous range as above) dealt
            // round-robin to its G/8 workgroups (G is a multiple of 8 here)
            const uint32_t g8 = gridDim.x / 8, x = blockIdx.x % 8;
            t0 = (a.ntiles * x) / 8 + blockIdx.x / 8;
            t1 = (a.ntiles * (x + 1)) / 8;
            tstep = g8;
        }
        load_masks(a.lp, a.nmodes, lmask);
        if (kUseLut<FAST, WORDS, LPN> && a.lut) build_nibble_lut(lmask, lut);
        mttkrp_stretch_pipe<LPN, FT, WORDS, MAXO, TMC, FAST, kOpMttkrp, FAST ? (F64 ? 2 : 1) : 0>(a, smem, nkeep, lmask,
                                                                                              t0, t1, lut, tstep);
    } else {
        mttkrp_stretch<LPN, FT, WORDS, MAXO, TMC>(a, smem, nkeep, t0, t1);
    }
}

// Many tensors in one persistent launch: the tiles of all jobs form one
// list (prefix[j] = first tile of job j); each workgroup drains a balanced
// stretch of it, crossing job boundaries.
template <int LPN, typename FT, int WORDS, int MAXO>
__global__ __launch_bounds__(512) void k_mttkrp_batch(const MttkrpArgs *__restrict__ jobs,
                                                      const uint64_t *__restrict__ prefix, int njobs, int xcd_map) {
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ uint32_t nkeep;
    __shared__ uint64_t lmask[MAXO <= 4 ? kMaskWords : 1];
    uint64_t g0, g1;
    stretch_of(prefix[njobs], xcd_map, &g0, &g1);
    // first job whose tiles reach past g0
    int lo = 0, hi = njobs;
    while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (prefix[mid + 1] <= g0) lo = mid + 1;
        else hi = mid;
    }
    for (int j = lo; j < njobs && prefix[j] < g1; j++) {
        const uint64_t a0 = prefix[j], a1 = prefix[j + 1];
        const uint64_t t0 = (g0 > a0 ? g0 : a0) - a0, t1 = (g1 < a1 ? g1 : a1) - a0;
        if (t0 < t1) {
            if constexpr (MAXO <= 4) {
                load_masks(jobs[j].lp, jobs[j].nmodes, lmask);
                mttkrp_stretch_pipe<LPN, FT, WORDS, MAXO, -1, false>(jobs[j], smem, nkeep, lmask, t0, t1);
            } else {
                mttkrp_stretch<LPN, FT, WORDS, MAXO, -1>(jobs[j], smem, nkeep, t0, t1);
            }
            __syncthreads();
        }
    }
}

// CP-APR model update Phi of one mode (OP kOpPhi or kOpPhiPre, see the
// pipelined stretch).
template <int LPN, int WORDS, int OP>
__global__ __launch_bounds__(512) void k_phi(const MttkrpArgs a) {
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ uint32_t nkeep;
    __shared__ uint64_t lmask[kMaskWords];
    uint64_t t0, t1;
    stretch_of(a.ntiles, a.xcd_map, &t0, &t1);
    load_masks(a.lp, a.nmodes, lmask);
    mttkrp_stretch_pipe<LPN, float, WORDS, 4, -1, false, OP>(a, smem, nkeep, lmask, t0, t1);
}

// Pi of one mode for the nonzeros (ALTO-PRE): row x of pi = Hadamard product
// of the other factors' rows at nonzero x, in ALTO order.  A group of LPN
// lanes per nonzero, 4 columns per lane; every lane de-linearizes the index.
template <int LPN, int WORDS>
__global__ __launch_bounds__(256) void k_phi_pi(const MttkrpArgs a, float *__restrict__ pi) {
    __shared__ uint64_t lmask[kMaskWords];
    load_masks(a.lp, a.nmodes, lmask);
    const int q = threadIdx.x & (LPN - 1);
    const int r0 = 4 * q;
    if (r0 >= a.rank) return;
    const uint64_t groups = (uint64_t)gridDim.x * (blockDim.x / LPN);
    for (uint64_t x = (uint64_t)blockIdx.x * (blockDim.x / LPN) + threadIdx.x / LPN; x < a.nnz; x += groups) {
        const uint64_t lo = a.keys[x * WORDS];
        const uint64_t hi = WORDS == 2 ? a.keys[x * WORDS + 1] : 0;
        float4 p = make_float4(1.f, 1.f, 1.f, 1.f);
        int k = 0;
        for (int m = 0; m < a.nmodes; m++) {
            if (m == a.mode) continue;
            const uint32_t i = min(extract_lds<WORDS>(lmask, m, lo, hi), a.last_other[k]);
            const float4 f = *(const float4 *)((const float *)a.fac_other[k] + (uint64_t)i * a.ld + r0);
            p.x *= f.x;
            p.y *= f.y;
            p.z *= f.z;
            p.w *= f.w;
            k++;
        }
        *(float4 *)(pi + x * a.ld + r0) = p;
    }
}

// Zero every job's output (grid-stride over the concatenated outputs).
__global__ void k_zero_outputs(const MttkrpArgs *__restrict__ jobs, const uint64_t *__restrict__ out_prefix,
                               int njobs) {
    const uint64_t total = out_prefix[njobs];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    int j = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        while (out_prefix[j + 1] <= i) j++;
        jobs[j].out32[i - out_prefix[j]] = 0.f;
    }
}

// out = FP32 rounding of the FP64 sum over `copies` partial outputs.
template <typename T>
__global__ void k_sum_copies(const T *__restrict__ in, int copies, uint64_t n, float *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double s = 0.0;
        for (int c = 0; c < copies; c++) s += (double)in[(uint64_t)c * n + i];
        out[i] = (float)s;
    }
}

// Kernel pointers for one factor type and index width (instantiated only in
// the unit that asks for them).
template <int LPN, typename FT, int WORDS>
const void *kernel_ptr(int nmodes, bool batch) {
    if (nmodes <= 3)
        return batch ? (const void *)k_mttkrp_batch<LPN, FT, WORDS, 2>
                     : (const void *)k_mttkrp<LPN, FT, WORDS, 2, -1, false>;
    if (nmodes <= 5)
        return batch ? (const void *)k_mttkrp_batch<LPN, FT, WORDS, 4>
                     : (const void *)k_mttkrp<LPN, FT, WORDS, 4, -1, false>;
    return batch ? (const void *)k_mttkrp_batch<LPN, FT, WORDS, 7> : (const void *)k_mttkrp<LPN, FT, WORDS, 7, -1, false>;
}

template <int LPN, typename FT, bool F64>
const void *fast_ptr(int tile_merge) {
    return tile_merge == 1   ? (const void *)k_mttkrp<LPN, FT, 1, 2, 1, true, F64>
           : tile_merge == 2 ? (const void *)k_mttkrp<LPN, FT, 1, 2, 2, true, F64>
           : tile_merge == 3 ? (const void *)k_mttkrp<LPN, FT, 1, 2, 3, true, F64>
                             : (const void *)k_mttkrp<LPN, FT, 1, 2, 0, true, F64>;
}

template <typename FT, bool F64>
const void *pick_fast(int lpn, int tile_merge) {
    switch (lpn) {
        case 1: return fast_ptr<1, FT, F64>(tile_merge);
        case 2: return fast_ptr<2, FT, F64>(tile_merge);
        case 4: return fast_ptr<4, FT, F64>(tile_merge);
        case 8: return fast_ptr<8, FT, F64>(tile_merge);
        case 16: return fast_ptr<16, FT, F64>(tile_merge);
        default: return fast_ptr<32, FT, F64>(tile_merge);
    }
}

template <int WORDS, int OP>
const void *phi_lpn(int lpn) {
    switch (lpn) {
        case 1: return (const void *)k_phi<1, WORDS, OP>;
        case 2: return (const void *)k_phi<2, WORDS, OP>;
        case 4: return (const void *)k_phi<4, WORDS, OP>;
        case 8: return (const void *)k_phi<8, WORDS, OP>;
        case 16: return (const void *)k_phi<16, WORDS, OP>;
        default: return (const void *)k_phi<32, WORDS, OP>;
    }
}

template <int WORDS>
const void *phi_pi_lpn(int lpn) {
    switch (lpn) {
        case 1: return (const void *)k_phi_pi<1, WORDS>;
        case 2: return (const void *)k_phi_pi<2, WORDS>;
        case 4: return (const void *)k_phi_pi<4, WORDS>;
        case 8: return (const void *)k_phi_pi<8, WORDS>;
        case 16: return (const void *)k_phi_pi<16, WORDS>;
        default: return (const void *)k_phi_pi<32, WORDS>;
    }
}

template <typename FT, int WORDS>
const void *pick_lpn(int lpn, int nmodes, bool batch) {
    switch (lpn) {
        case 1: return kernel_ptr<1, FT, WORDS>(nmodes, batch);
        case 2: return kernel_ptr<2, FT, WORDS>(nmodes, batch);
        case 4: return kernel_ptr<4, FT, WORDS>(nmodes, batch);
        case 8: return kernel_ptr<8, FT, WORDS>(nmodes, batch);
        case 16: return kernel_ptr<16, FT, WORDS>(nmodes, batch);
        default: return kernel_ptr<32, FT, WORDS>(nmodes, batch);
    }
}


}  // namespace

}  // namespace alto
