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
#include <string.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "alto_internal.h"
#include "device_util.h"
#include "memory.h"
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

// Hardware id of the XCD (accelerator complex die) running this wave.
__device__ inline uint32_t xcd_id() { return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & 15u; }

// Add 4 columns of partial sums (FP32 run sums or FP64 LDS rows) to the
// output row, or to this XCD's copy of it.
// FAST: the plan is known to add FP32 straight into the output.
template <bool FAST = false, typename T>
__device__ inline void global_add(const MttkrpArgs &a, uint32_t row, int r0, const T *acc) {
    uint64_t o = (uint64_t)row * a.ld + a.col0 + r0;
    if (FAST) {
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (r0 + j < a.rank) unsafeAtomicAdd(a.out32 + o + j, (float)acc[j]);
        return;
    }
    if (a.copies > 1) o += (uint64_t)(xcd_id() % (uint32_t)a.copies) * a.copy_stride;
    if (a.use64) {
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (r0 + j < a.rank) unsafeAtomicAdd(a.out64 + o + j, (double)acc[j]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (r0 + j < a.rank) unsafeAtomicAdd(a.out32 + o + j, (float)acc[j]);
    }
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
template <int TM, bool FAST>
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
        global_add<FAST>(a, dst, r0, acc);
    }
}

constexpr uint32_t kFlushMark = 0xFFFFFFFFu;

// Coordinate k of the other modes from a staged record held as two uint4.
__device__ inline uint32_t rec_coord(const uint4 &h, const uint4 &h2, int k) {
    return k == 0 ? h.z : k == 1 ? h.w : k == 2 ? h2.x : k == 3 ? h2.y : k == 4 ? h2.z : h2.w;
}

// Kernel variants: MAXO = most other modes handled with fully unrolled
// gathers (2: up to 3-mode tensors, 4: up to 5 modes); 7: any order, rolled.
// End of tile t of the stretch [t0, t1): the LDS table's rows go to the
// output -- for a whole-mode table (TM 2) once, at the stretch's end; for a
// hashed table (TM 1) every tile, except rows merged many times (high
// reuse), which stay for the next tile.  Everything is flushed every
// kKeepTiles tiles and at the end of the stretch.
template <bool FAST>
__device__ inline void tile_end(const MttkrpArgs &a, int TM, int TW, int S, int TS, uint32_t *tkey, uint32_t *thits,
                                void *tval, uint32_t &nkeep, uint64_t t, uint64_t t0, uint64_t t1) {
    const int tid = threadIdx.x;
    double *tv64 = (double *)tval;
    float *tv32 = (float *)tval;
    if (TM == 2 && t + 1 == t1) {
        // ---- end of the stretch: every row of the mode held in LDS is
        // added to the output once
        __syncthreads();
        const int qr = a.rank >> 2;
        for (int i = tid; i < S * qr; i += blockDim.x) {
            const int row = i / qr, part = i - row * qr;
            if (TW == 2) {
                const double *tv = tv64 + (size_t)row * TS + part * 4;
                const double vv[4] = {tv[0], tv[1], tv[2], tv[3]};
                if (vv[0] != 0.0 || vv[1] != 0.0 || vv[2] != 0.0 || vv[3] != 0.0)
                    global_add<FAST>(a, (uint32_t)row, part * 4, vv);
            } else {
                const float *tv = tv32 + (size_t)row * TS + part * 4;
                const float vv[4] = {tv[0], tv[1], tv[2], tv[3]};
                if (vv[0] != 0.f || vv[1] != 0.f || vv[2] != 0.f || vv[3] != 0.f)
                    global_add<FAST>(a, (uint32_t)row, part * 4, vv);
            }
        }
        __syncthreads();
    } else if (TM == 1) {
        __syncthreads();
        const bool flush_all = (t + 1 == t1) || ((t - t0 + 1) % kKeepTiles == 0);
        if (tid == 0) nkeep = 0;
        __syncthreads();
        for (int i = tid; i < S; i += blockDim.x) {
            if (tkey[i] == kEmptyRow) continue;
            bool keep = false;
            if (!flush_all && thits[i] >= kHotHits) keep = atomicAdd(&nkeep, 1u) < (uint32_t)(S / 4);
            thits[i] = keep ? 0u : kFlushMark;
        }
        __syncthreads();
        const int qr = a.rank >> 2;
        for (int i = tid; i < S * qr; i += blockDim.x) {
            const int slot = i / qr, part = i - slot * qr;
            if (thits[slot] == kFlushMark) {
                double *tv = tv64 + (size_t)slot * TS + part * 4;
                const double vv[4] = {tv[0], tv[1], tv[2], tv[3]};
                global_add<FAST>(a, tkey[slot], part * 4, vv);
                tv[0] = 0.0;
                tv[1] = 0.0;
                tv[2] = 0.0;
                tv[3] = 0.0;
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
// plain, unpipelined loop: single launches of shapes other than the
// specialised one, and tensors of 6-8 modes in batched launches).  The LDS
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

        tile_end<false>(a, TM, TW, S, TS, tkey, thits, tval, nkeep, t, t0, t1);
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

// Coordinate of mode m from an index (lo, hi) with the masks in LDS.
template <int WORDS>
__device__ inline uint32_t extract_lds(const uint64_t *lm, int m, uint64_t lo, uint64_t hi) {
    const uint64_t *mm = lm + m * kMaskStride;
    uint64_t c = compress_lds(lo, mm);
    if (WORDS == 2) c |= compress_lds(hi, mm + 7) << (uint32_t)mm[14];
    return (uint32_t)c;
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
// modes, one-word index, 32-bit buffer gathers and FP32 atomics into the
// output (the specialised kernel).
template <int LPN, typename FT, int WORDS, int MAXO, int TMC, bool FAST>
__device__ inline void mttkrp_stretch_pipe(const MttkrpArgs &a, uint32_t *smem, uint32_t &nkeep,
                                           const uint64_t *lmask, uint64_t t0, uint64_t t1) {
    static_assert(MAXO == 2 || MAXO == 4, "pipelined stretch: up to 5 modes");
    const int TM = TMC >= 0 ? TMC : a.tile_merge;
    constexpr int SB = MAXO == 2 ? (LPN < 4 ? LPN : 4) : (LPN < 2 ? LPN : 2);  // records per step
    constexpr int NS = LPN / SB;                                               // steps per batch
    constexpr int RW = MAXO == 2 ? 4 : 8;                                      // record words
    const int nmodes = FAST ? 3 : a.nmodes;
    const int nother = nmodes - 1;
    const int S = TM == 1 ? (1 << a.slots_log2) : (TM == 2 ? (int)a.dim_out : 0);
    const int SK = TM == 1 ? S : 0;
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
    __amdgpu_buffer_rsrc_t rs[MAXO];
#pragma unroll
    for (int k = 0; k < MAXO; k++)
        if (k < nother) rs[k] = factor_rsrc(a.fac_other[k], a.fac_bytes[k]);
    const uint32_t ldb = a.ld * (uint32_t)sizeof(FT);
    const uint32_t colb = (a.col0 + (uint32_t)r0) * (uint32_t)sizeof(FT);
    const int mode = a.mode;

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
#pragma unroll
                for (int m = 0; m <= MAXO; m++) c[m] = m < nmodes ? extract_lds<WORDS>(lmask, m, lo, hi) : 0u;
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
                    }
                    r[0] = __float_as_uint(val);
                    r[1] = dst;
#pragma unroll
                    for (int k = 0; k < MAXO; k++) r[2 + k] = k < mode ? c[k] : c[k + 1];
                }
            }
            uint32_t *rec = gbuf + q * RW;
            *(uint4 *)rec = make_uint4(r[0], r[1], r[2], r[3]);
            if (RW == 8) *(uint4 *)(rec + 4) = make_uint4(r[4], r[5], r[6], r[7]);
        };
        // step k: its records' heads, and the gathers of the other modes
        auto issue = [&](uint64_t k, float4 (&g)[MAXO][SB], uint32_t (&dv)[SB], float (&vv)[SB]) {
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
#pragma unroll
                for (int k2 = 0; k2 < MAXO; k2++) {
                    if (k2 < nother) {
                        if (buf32) {
                            g[k2][s] = bload4<FT>(rs[k2], idx[k2] * ldb + colb);
                        } else {
                            const uint32_t ii = min(idx[k2], a.last_other[k2]);
                            g[k2][s] = ract ? load4<FT>(a.fac_other[k2], (uint64_t)ii * a.ld + a.col0 + r0)
                                            : make_float4(0.f, 0.f, 0.f, 0.f);
                        }
                    }
                }
            }
        };
        // products of a step, merged into runs of equal destinations
        auto consume = [&](const float4 (&g)[MAXO][SB], const uint32_t (&dv)[SB], const float (&vv)[SB]) {
#pragma unroll
            for (int s = 0; s < SB; s++) {
                if (dv[s] == kEmptyRow) continue;
                float p[4] = {vv[s], vv[s], vv[s], vv[s]};
#pragma unroll
                for (int k2 = 0; k2 < MAXO; k2++) {
                    if (k2 < nother) {
                        p[0] *= g[k2][s].x;
                        p[1] *= g[k2][s].y;
                        p[2] *= g[k2][s].z;
                        p[3] *= g[k2][s].w;
                    }
                }
                if (dv[s] == cur) {
#pragma unroll
                    for (int j = 0; j < 4; j++) acc[j] += p[j];
                } else {
                    if (cur != kEmptyRow) flush_run<TMC, FAST>(a, tval, thits, cur, q, r0, acc);
                    cur = dv[s];
#pragma unroll
                    for (int j = 0; j < 4; j++) acc[j] = p[j];
                }
            }
        };

        float4 xg[MAXO][SB], yg[MAXO][SB];
        uint32_t xd[SB], yd[SB];
        float xv[SB], yv[SB];
        if (nsteps > 0) issue(0, xg, xd, xv);
        for (uint64_t k = 0; k < nsteps; k += 2) {
            if (k + 1 < nsteps) issue(k + 1, yg, yd, yv);
            consume(xg, xd, xv);
            if (k + 1 >= nsteps) break;
            if (k + 2 < nsteps) issue(k + 2, xg, xd, xv);
            consume(yg, yd, yv);
        }
        if (cur != kEmptyRow) flush_run<TMC, FAST>(a, tval, thits, cur, q, r0, acc);
        __builtin_amdgcn_wave_barrier();
        tile_end<FAST>(a, TM, TW, S, TS, tkey, thits, tval, nkeep, t, t0, t1);
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
template <int LPN, typename FT, int WORDS, int MAXO, int TMC, bool FAST>
__global__ __launch_bounds__(512) void k_mttkrp(const MttkrpArgs a) {
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ uint32_t nkeep;
    __shared__ uint64_t lmask[FAST ? kMaskWords : 1];
    uint64_t t0, t1;
    stretch_of(a.ntiles, a.xcd_map, &t0, &t1);
    // single launches: the pipelined loop for the specialised case; for
    // other shapes it measured slower than the plain loop (more registers
    // and scalar state per step), while it pays in the batched launches
    if constexpr (FAST) {
        load_masks(a.lp, a.nmodes, lmask);
        mttkrp_stretch_pipe<LPN, FT, WORDS, MAXO, TMC, FAST>(a, smem, nkeep, lmask, t0, t1);
    } else {
        mttkrp_stretch<LPN, FT, WORDS, MAXO, TMC>(a, smem, nkeep, t0, t1);
    }
}

// Many tensors in one persistent launch: the tiles of all jobs form one
// list (prefix[j] = first tile of job j); each workgroup drains a balanced
// stretch of it, crossing job boundaries.
template <int LPN, typename FT, int WORDS, int MAXO>
__global__ __launch_bounds__(256, 2) void k_mttkrp_batch(const MttkrpArgs *__restrict__ jobs,
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

template <int LPN, typename FT>
const void *fast_ptr(int tile_merge) {
    return tile_merge == 1   ? (const void *)k_mttkrp<LPN, FT, 1, 2, 1, true>
           : tile_merge == 2 ? (const void *)k_mttkrp<LPN, FT, 1, 2, 2, true>
                             : (const void *)k_mttkrp<LPN, FT, 1, 2, 0, true>;
}

template <typename FT>
const void *pick_fast(int lpn, int tile_merge) {
    switch (lpn) {
        case 1: return fast_ptr<1, FT>(tile_merge);
        case 2: return fast_ptr<2, FT>(tile_merge);
        case 4: return fast_ptr<4, FT>(tile_merge);
        case 8: return fast_ptr<8, FT>(tile_merge);
        case 16: return fast_ptr<16, FT>(tile_merge);
        default: return fast_ptr<32, FT>(tile_merge);
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

const void *pick_kernel(int lpn, int fdt, int words, int nmodes, bool batch) {
    if (fdt == ALTO_BF16)
        return words == 2 ? pick_lpn<uint16_t, 2>(lpn, nmodes, batch) : pick_lpn<uint16_t, 1>(lpn, nmodes, batch);
    return words == 2 ? pick_lpn<float, 2>(lpn, nmodes, batch) : pick_lpn<float, 1>(lpn, nmodes, batch);
}

// The specialised kernel serves 3-mode tensors with a one-word index whose
// factor reads fit 32-bit offsets and whose updates go straight to the FP32
// output; everything else takes the general kernel.
const void *pick_single(int lpn, int fdt, int words, const MttkrpArgs &a) {
    if (words == 1 && a.nmodes == 3 && a.buf32 && !a.use64 && a.copies == 1)
        return fdt == ALTO_BF16 ? pick_fast<uint16_t>(lpn, a.tile_merge) : pick_fast<float>(lpn, a.tile_merge);
    return pick_kernel(lpn, fdt, words, a.nmodes, false);
}

const void *zero_outputs_kernel() { return (const void *)k_zero_outputs; }

namespace {

struct DevProps {
    int cus = 0;
    size_t lds = 0;  // LDS bytes one workgroup may allocate
};

DevProps &props(int dev);
}  // namespace

int device_cus(int dev) { return props(dev).cus; }

// Static LDS of the MTTKRP kernels (extraction masks, counters) is below
// this; plans budget it beside their tables and record staging.
constexpr size_t kStaticLdsAllowance = 2048;

// LDS words staged per nonzero: [value, destination, other coordinates]
// rounded to 16 bytes.
int record_words(int nmodes, int words) {
    (void)words;
    return (nmodes + 1 + 3) / 4 * 4;
}

size_t tile_plan_lds(const alto_tensor *h, int rank_tile, int slots, int threads) {
    const size_t rec = (size_t)record_words(h->info.nmodes, h->info.index_words);
    return (size_t)slots * (2 * (rank_tile + 1) + 2) * 4 + (size_t)threads * rec * 4 + kStaticLdsAllowance;
}

bool tile_plan_fits(const alto_tensor *h, int rank_tile, int slots, int threads) {
    return tile_plan_lds(h, rank_tile, slots, threads) <= props(h->device).lds;
}

alto_status check_launch_lds(const void *kern, size_t dyn, int dev) {
    hipFuncAttributes fa;
    size_t stat = 256;
    if (hipFuncGetAttributes(&fa, kern) == hipSuccess) stat = fa.sharedSizeBytes;
    else (void)hipGetLastError();
    if (dyn + stat > props(dev).lds)
        return fail(ALTO_ERR_ARG, "launch needs " + std::to_string(dyn + stat) + " bytes of LDS; the device has " +
                                      std::to_string(props(dev).lds));
    return ALTO_OK;
}

size_t direct_table_limit(const alto_tensor *h, int threads) {
    const size_t rec = (size_t)record_words(h->info.nmodes, h->info.index_words);
    const size_t stage = (size_t)threads * rec * 4 + kStaticLdsAllowance;  // + static LDS and alignment
    const size_t lds = props(h->device).lds;
    return lds > stage ? lds - stage : 0;
}

namespace {

DevProps &props(int dev) {
    static DevProps p[64];
    if (dev >= 0 && dev < 64 && p[dev].cus == 0) {
        hipDeviceProp_t dp;
        if (hipGetDeviceProperties(&dp, dev) == hipSuccess) {
            p[dev].cus = dp.multiProcessorCount;
            p[dev].lds = dp.sharedMemPerBlock;
        } else {
            p[dev].cus = 256;
            p[dev].lds = 64 * 1024;
        }
    }
    return p[dev < 0 || dev >= 64 ? 0 : dev];
}

}  // namespace

int pow2_floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

int lpn_for(int rank) {
    int l = 1;
    while (4 * l < rank) l <<= 1;
    return l;
}

alto_mttkrp_plan default_plan(const alto_tensor *h, int mode, int rank, int fdt) {
    alto_mttkrp_plan p;
    memset(&p, 0, sizeof(p));
    const double reuse = (double)h->info.nnz / (double)h->info.dims[mode];
    // initial rule of the paper: buffered (tile) merging pays off when the
    // average number of nonzeros per output fiber exceeds the 4 memory
    // operations a buffered update costs in the worst case
    p.conflict = reuse > 4.0 ? ALTO_CR_TILE : ALTO_CR_RUN;
    p.block_threads = 256;
    // LDS table of about 64 KiB of FP64 partial rows
    int slots = 8192 / rank;
    int s2 = 1;
    while (s2 * 2 <= slots) s2 *= 2;
    p.table_slots = std::max(64, s2);
    // long tiles amortize the table flush; keep enough tiles to fill the GPU
    uint64_t tile = 512;
    while (tile < 16384 && tile * 8192 < h->info.nnz) tile *= 2;
    p.tile_nnz = (int)tile;
    p.accumulate = ALTO_ACC_F32;
    // a mode short enough to hold whole in LDS (with a rank tile of at least
    // 8 columns) is accumulated there for the workgroup's whole segment: in
    // FP64 rows if at most two passes (rank tiles) do, else in FP32 rows
    // (twice the columns per pass, slower adds)
    const size_t lim = direct_table_limit(h, 512);
    int rt_d = 0;
    size_t bytes_d = 0;
    for (int eb : {8, 4}) {
        for (int rt = rank; rt >= 8 && rt % 4 == 0 && rank % rt == 0; rt /= 2) {
            const size_t bytes = (size_t)h->info.dims[mode] * (rt + 1) * eb;
            if (bytes <= lim) {
                if (eb == 4 || 2 * rt >= rank) {
                    rt_d = rt;
                    bytes_d = bytes;
                }
                break;
            }
        }
        if (rt_d) break;
    }
    if (rt_d && reuse > 4.0) {
        p.conflict = ALTO_CR_DIRECT;
        p.rank_tile = rt_d == rank ? 0 : rt_d;
        // one workgroup per CU when the table takes most of the LDS: give it
        // more waves
        if (bytes_d > direct_table_limit(h, 256) / 2) p.block_threads = 512;
    }
    (void)fdt;
    return p;
}

static std::mutex g_tune_mu;
static std::map<std::array<int, 6>, alto_mttkrp_plan> g_tune_cache;

std::array<int, 6> tune_key(const alto_tensor *h, int mode, int rank, int fdt) {
    const double reuse = (double)h->info.nnz / (double)h->info.dims[mode];
    const int lr = reuse > 0 ? (int)std::floor(std::log2(reuse)) : -64;
    const int ln = h->info.nnz > 0 ? (int)std::floor(std::log2((double)h->info.nnz)) : -1;
    return {h->info.nmodes, rank, h->info.index_words, fdt, lr, ln};
}

void record_tuned(alto_tensor *h, int mode, int rank, int fdt, const alto_mttkrp_plan &p) {
    h->tuned[mode][fdt][rank / 4] = p;
    h->has_tuned[mode][fdt][rank / 4] = true;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[tune_key(h, mode, rank, fdt)] = p;
}

bool cached_tuned(const alto_tensor *h, int mode, int rank, int fdt, alto_mttkrp_plan *p) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(tune_key(h, mode, rank, fdt));
    if (it == g_tune_cache.end()) return false;
    *p = it->second;
    return true;
}

alto_status resolve_plan(const alto_tensor *h, int mode, int rank, int fdt, const alto_mttkrp_plan *in,
                         alto_mttkrp_plan *out) {
    alto_mttkrp_plan p = default_plan(h, mode, rank, fdt);
    const int ri = rank / 4;
    if (ri >= 0 && ri <= 32 && h->has_tuned[mode][fdt][ri]) p = h->tuned[mode][fdt][ri];
    else if (ri >= 0 && ri <= 32) cached_tuned(h, mode, rank, fdt, &p);
    if (in) {
        if (in->conflict) {
            p.conflict = in->conflict;
            p.rank_tile = 0;
        }
        if (in->rank_tile) p.rank_tile = in->rank_tile;
        if (in->tile_nnz) p.tile_nnz = in->tile_nnz;
        if (in->block_threads) p.block_threads = in->block_threads;
        if (in->table_slots) p.table_slots = in->table_slots;
        if (in->accumulate) p.accumulate = in->accumulate;
    }
    if (p.accumulate < ALTO_ACC_F64 || p.accumulate > ALTO_ACC_XCD_F64) return fail(ALTO_ERR_ARG, "bad accumulate mode");
    if (p.conflict != ALTO_CR_TILE && p.conflict != ALTO_CR_RUN && p.conflict != ALTO_CR_DIRECT)
        return fail(ALTO_ERR_ARG, "bad conflict mode");
    if (p.rank_tile < 0 || p.rank_tile % 4 || (p.rank_tile > 0 && rank % p.rank_tile))
        return fail(ALTO_ERR_ARG, "rank_tile must be a multiple of 4 dividing rank");
    const int rt = p.rank_tile > 0 ? p.rank_tile : rank;
    if (p.block_threads != 256 && p.block_threads != 512) return fail(ALTO_ERR_ARG, "block_threads must be 256 or 512");
    if (p.conflict == ALTO_CR_DIRECT &&
        (size_t)h->info.dims[mode] * (rt + 1) * 4 > direct_table_limit(h, p.block_threads))
        return fail(ALTO_ERR_ARG, "mode too long to hold in LDS for this rank tile");
    if (p.tile_nnz < 1) return fail(ALTO_ERR_ARG, "tile_nnz must be positive");
    if (p.conflict == ALTO_CR_TILE) {
        if (p.table_slots < 16 || (p.table_slots & (p.table_slots - 1)))
            return fail(ALTO_ERR_ARG, "table_slots must be a power of two >= 16");
        // FP64 rows + keys + hit counts, the record staging and static LDS
        if (!tile_plan_fits(h, rt, p.table_slots, p.block_threads))
            return fail(ALTO_ERR_ARG, "LDS table too large for rank and block size");
    }
    *out = p;
    return ALTO_OK;
}

alto_status check_mttkrp_args(const alto_tensor *h, int mode, int rank, int fdt, const void *const *factors,
                              const float *out) {
    ALTO_CHECK_HANDLE(h);
    if (mode < 0 || mode >= h->info.nmodes) return fail(ALTO_ERR_ARG, "mode out of range");
    if (rank < 4 || rank > ALTO_MAX_RANK || rank % 4) return fail(ALTO_ERR_ARG, "rank must be a multiple of 4 in 4..128");
    if (fdt != ALTO_F32 && fdt != ALTO_BF16) return fail(ALTO_ERR_ARG, "bad factor dtype");
    if (!out) return fail(ALTO_ERR_ARG, "out is NULL");
    if (((uintptr_t)out & 15) != 0) return fail(ALTO_ERR_ARG, "out must be 16-byte aligned");
    if (!factors) return fail(ALTO_ERR_ARG, "factors is NULL");
    const uintptr_t al = fdt == ALTO_F32 ? 15 : 7;
    for (int m = 0; m < h->info.nmodes; m++) {
        if (m == mode) continue;
        if (!factors[m]) return fail(ALTO_ERR_ARG, "factors[" + std::to_string(m) + "] is NULL");
        if ((uintptr_t)factors[m] & al) return fail(ALTO_ERR_ARG, "factor rows must be 16-byte (8 for BF16) aligned");
    }
    return ALTO_OK;
}

alto_status ensure_ws(void **p, size_t *have, size_t need) {
    if (*have >= need && *p) return ALTO_OK;
    if (*p) {
        ALTO_HIP(hipDeviceSynchronize());
        dev_free(*p);
        *p = nullptr;
        *have = 0;
    }
    if (dev_alloc(p, need) != hipSuccess) return fail(ALTO_ERR_OOM, "workspace allocation failed");
    *have = need;
    return ALTO_OK;
}

void fill_args(const alto_tensor *h, int mode, int rank, int fdt, const void *const *factors,
               const alto_mttkrp_plan &p, float *out32, double *out64, MttkrpArgs *a, int col0, int rank_tile) {
    memset(a, 0, sizeof(*a));
    a->lp = h->lp;
    int k = 0;
    for (int m = 0; m < h->info.nmodes; m++)
        if (m != mode) {
            a->last_other[k] = (uint32_t)(h->info.dims[m] - 1);
            a->fac_other[k++] = factors[m];
        }
    a->dim_out = (uint32_t)h->info.dims[mode];
    // 32-bit buffer offsets reach every factor row when each factor is below 2 GiB
    const int fbytes = fdt == ALTO_BF16 ? 2 : 4;
    a->buf32 = 1;
    k = 0;
    for (int m = 0; m < h->info.nmodes; m++) {
        if (m == mode) continue;
        const uint64_t bytes = h->info.dims[m] * (uint64_t)rank * fbytes;
        if (bytes >= (uint64_t(1) << 31)) a->buf32 = 0;
        a->fac_bytes[k++] = (uint32_t)(bytes < (uint64_t(1) << 31) ? bytes : 0);
    }
    a->keys = h->keys;
    a->vals = h->vals;
    a->out32 = out32;
    a->out64 = out64;
    a->nnz = h->info.nnz;
    uint64_t L = (h->info.nnz + p.tile_nnz - 1) / p.tile_nnz;
    if (L < 1) L = 1;
    a->ntiles = L;
    a->tq = h->info.nnz / L;
    a->tr = h->info.nnz % L;
    a->mode = mode;
    a->rank = rank_tile > 0 ? rank_tile : rank;
    a->ld = (uint32_t)rank;
    a->col0 = (uint32_t)col0;
    a->nmodes = h->info.nmodes;
    a->tile_merge = p.conflict == ALTO_CR_TILE ? 1 : (p.conflict == ALTO_CR_DIRECT ? 2 : 0);
    a->use64 = (p.accumulate == ALTO_ACC_F64 || p.accumulate == ALTO_ACC_XCD_F64) ? 1 : 0;
    a->copies = (p.accumulate == ALTO_ACC_XCD_F32 || p.accumulate == ALTO_ACC_XCD_F64) ? kXcdCopies : 1;
    a->copy_stride = h->info.dims[mode] * (uint64_t)rank;
    int l2 = 0;
    while ((1 << l2) < p.table_slots) l2++;
    a->slots_log2 = l2;
    a->rec = record_words(h->info.nmodes, h->info.index_words);
    // whole-mode rows are FP64 when this rank tile fits so, else FP32
    a->tw = 2;
    if (a->tile_merge == 2 &&
        (size_t)h->info.dims[mode] * (a->rank + 1) * 8 > direct_table_limit(h, p.block_threads))
        a->tw = 1;
}

size_t lds_bytes(const MttkrpArgs &a, int threads) {
    const size_t S = a.tile_merge == 1 ? ((size_t)1 << a.slots_log2) : (a.tile_merge == 2 ? a.dim_out : 0);
    const size_t SK = a.tile_merge == 1 ? S : 0;
    const size_t TW = a.tile_merge == 2 ? (size_t)a.tw : 2;  // words per table element
    return ((2 * SK + TW * S * (a.rank + 1) + 3) & ~(size_t)3) * 4 + (size_t)threads * a.rec * 4;
}

// ---- optional per-launch timing with HIP events
namespace {
struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> pool;
};
Timing &timing() {
    static Timing *t = new Timing();
    return *t;
}
hipEvent_t take_event(Timing &t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}
void clear_pending(Timing &t) {
    for (auto &pr : t.pending) {
        (void)hipEventSynchronize(pr.second);
        t.pool.push_back(pr.first);
        t.pool.push_back(pr.second);
    }
    t.pending.clear();
}
}  // namespace

bool timing_begin(hipStream_t s, hipEvent_t *e0, hipEvent_t *e1) {
    Timing &t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.on) return false;
    *e0 = take_event(t);
    *e1 = take_event(t);
    if (!*e0 || !*e1) return false;
    (void)hipEventRecord(*e0, s);
    return true;
}

void timing_end(hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    Timing &t = timing();
    (void)hipEventRecord(e1, s);
    std::lock_guard<std::mutex> lk(t.mu);
    t.pending.push_back({e0, e1});
}

alto_status launch_mttkrp(const alto_tensor *h, int fdt, const MttkrpArgs &a, int threads, hipStream_t s) {
    const int lpn = lpn_for(a.rank);
    const void *kern = pick_single(lpn, fdt, h->info.index_words, a);
    const size_t lds = lds_bytes(a, threads);
    // never dispatch more LDS than a workgroup may hold
    alto_status lst = check_launch_lds(kern, lds, h->device);
    if (lst != ALTO_OK) return lst;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, lds) != hipSuccess || occ < 1) {
        (void)hipGetLastError();
        occ = 1;
    }
    const int cus = props(h->device).cus;
    uint64_t grid = (uint64_t)cus * occ;
    MttkrpArgs b = a;
    if (grid >= a.ntiles) {
        grid = a.ntiles;
        b.xcd_map = 0;
    } else {
        grid = grid / 8 * 8;
        b.xcd_map = 1;
    }
    if (grid < 1) grid = 1;
    void *args[] = {(void *)&b};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = timing_begin(s, &e0, &e1);
    ALTO_HIP(hipLaunchKernel(kern, dim3((unsigned)grid), dim3(threads), args, lds, s));
    if (timed) timing_end(s, e0, e1);
    return ALTO_OK;
}

alto_status run_mttkrp(alto_tensor *h, int mode, int rank, int fdt, const void *const *factors, float *out,
                       const alto_mttkrp_plan &p, hipStream_t s) {
    const uint64_t nout = h->info.dims[mode] * (uint64_t)rank;
    const bool f64 = p.accumulate == ALTO_ACC_F64 || p.accumulate == ALTO_ACC_XCD_F64;
    const int copies = (p.accumulate == ALTO_ACC_XCD_F32 || p.accumulate == ALTO_ACC_XCD_F64) ? kXcdCopies : 1;
    const bool direct = p.accumulate == ALTO_ACC_F32;  // atomics straight into `out`
    const unsigned g = grid_for(nout * copies, 256, 16384);
    double *out64 = nullptr;
    float *acc32 = out;
    if (!direct) {
        alto_status st = ensure_ws(&h->ws_acc, &h->ws_acc_bytes, nout * copies * (f64 ? 8 : 4));
        if (st != ALTO_OK) return st;
        if (f64) {
            out64 = (double *)h->ws_acc;
            hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(256), 0, s, out64, nout * copies, 0.0);
        } else {
            acc32 = (float *)h->ws_acc;
            hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(256), 0, s, acc32, nout * copies, 0.f);
        }
    } else {
        hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(256), 0, s, out, nout, 0.f);
    }
    ALTO_HIP(hipGetLastError());
    if (h->info.nnz > 0) {
        // one launch per rank tile (columns [c, c + rt) of factors and output)
        const int rt = p.rank_tile > 0 ? p.rank_tile : rank;
        for (int c = 0; c < rank; c += rt) {
            MttkrpArgs a;
            fill_args(h, mode, rank, fdt, factors, p, acc32, out64, &a, c, rt);
            alto_status st = launch_mttkrp(h, fdt, a, p.block_threads, s);
            if (st != ALTO_OK) return st;
        }
    }
    if (!direct) {
        const unsigned g1 = grid_for(nout, 256, 16384);
        if (f64) hipLaunchKernelGGL(k_sum_copies<double>, dim3(g1), dim3(256), 0, s, out64, copies, nout, out);
        else hipLaunchKernelGGL(k_sum_copies<float>, dim3(g1), dim3(256), 0, s, acc32, copies, nout, out);
        ALTO_HIP(hipGetLastError());
    }
    return ALTO_OK;
}

}  // namespace alto

using namespace alto;

extern "C" {

alto_status alto_mttkrp_ex(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors, float *out,
                           const alto_mttkrp_plan *plan, void *stream) {
    alto_status st = check_mttkrp_args(h, mode, rank, fdt, factors, out);
    if (st != ALTO_OK) return st;
    alto_mttkrp_plan p;
    st = resolve_plan(h, mode, rank, fdt, plan, &p);
    if (st != ALTO_OK) return st;
    return run_mttkrp(h, mode, rank, fdt, factors, out, p, (hipStream_t)stream);
}

alto_status alto_mttkrp(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors, float *out,
                        void *stream) {
    return alto_mttkrp_ex(h, mode, rank, fdt, factors, out, nullptr, stream);
}

alto_status alto_timing_enable(int on) {
    Timing &t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    clear_pending(t);
    t.on = on != 0;
    return ALTO_OK;
}

alto_status alto_timing_read(uint64_t *launches, double *total_ms) {
    if (!launches || !total_ms) return fail(ALTO_ERR_ARG, "NULL argument");
    Timing &t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    double tot = 0.0;
    for (auto &pr : t.pending) {
        float ms = 0.f;
        ALTO_HIP(hipEventSynchronize(pr.second));
        ALTO_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        tot += ms;
    }
    *launches = t.pending.size();
    *total_ms = tot;
    clear_pending(t);
    return ALTO_OK;
}

alto_status alto_release_cached_memory(void) {
    ALTO_HIP(hipDeviceSynchronize());
    release_cached();
    return ALTO_OK;
}

alto_status alto_mttkrp_get_plan(alto_handle h, int mode, int rank, alto_dtype fdt, alto_mttkrp_plan *out) {
    ALTO_CHECK_HANDLE(h);
    if (!out) return fail(ALTO_ERR_ARG, "out is NULL");
    if (mode < 0 || mode >= h->info.nmodes) return fail(ALTO_ERR_ARG, "mode out of range");
    if (rank < 4 || rank > ALTO_MAX_RANK || rank % 4) return fail(ALTO_ERR_ARG, "rank must be a multiple of 4 in 4..128");
    if (fdt != ALTO_F32 && fdt != ALTO_BF16) return fail(ALTO_ERR_ARG, "bad factor dtype");
    return resolve_plan(h, mode, rank, fdt, nullptr, out);
}

}  // extern "C"
