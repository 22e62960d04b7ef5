// Autotuning of the MTTKRP launch plan and batched MTTKRP.
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "alto_internal.h"
#include "device_util.h"
#include "memory.h"
#include "mttkrp.h"

namespace alto {
namespace {

struct Group {
    int lpn, fdt, words, maxo;
    std::vector<int> items;
};

// Launch plan of a group: tile length, LDS table rows (quarters of the
// single-tensor default), threads per workgroup.
using BatchPlan = std::array<int, 3>;

int maxo_of(int nmodes) { return nmodes <= 3 ? 2 : (nmodes <= 5 ? 4 : 7); }

// Host side of one group's persistent launch: the per-job kernel arguments,
// tile and output prefixes, LDS size and kernel.
alto_status plan_group(const Group &g, const alto_handle *hs, const int *modes, const int *ranks,
                       const void *const *const *factors, float *const *outs, const BatchPlan &bp,
                       hipStream_t s, int dev, GroupLaunch *gl) {
    const int nj = (int)g.items.size();
    const int tile = bp[0], slots_factor = bp[1], threads = bp[2];
    gl->nj = nj;
    gl->threads = threads;
    gl->jobs.assign(nj, MttkrpArgs{});
    gl->prefix.assign(nj + 1, 0);
    gl->oprefix.assign(nj + 1, 0);
    size_t lds = 0;
    // one tile length for every job of the launch (at least each job's
    // nnz / kBatchF32MaxTiles), so that equal tile counts are equal work
    uint64_t tlen = (uint64_t)tile;
    for (int k = 0; k < nj; k++)
        tlen = std::max<uint64_t>(tlen, (hs[g.items[k]]->info.nnz + kBatchF32MaxTiles - 1) / kBatchF32MaxTiles);
    for (int k = 0; k < nj; k++) {
        const int j = g.items[k];
        alto_tensor *h = hs[j];
        h->stream = s;
        alto_mttkrp_plan p = default_plan(h, modes[j], ranks[j], g.fdt);
        p.conflict = ALTO_CR_TILE;
        p.rank_tile = 0;
        p.accumulate = ALTO_ACC_F32;
        // FP32 atomics into the output: a row takes at most one addition per
        // tile, so long tensors get longer tiles (see accuracy_policy)
        p.tile_nnz = (int)tlen;
        // table rows: slots_factor quarters of the single-tensor default
        p.table_slots = std::max(16, p.table_slots * slots_factor / 4);
        // one LDS size serves the whole launch: keep every table within
        // 96 KiB of FP64 rows, keys and hit counts
        while (p.table_slots > 16 && (size_t)p.table_slots * (2 * (ranks[j] + 1) + 2) * 4 > 96 * 1024)
            p.table_slots /= 2;
        fill_args(h, modes[j], ranks[j], g.fdt, factors[j], p, outs[j], nullptr, &gl->jobs[k]);
        gl->jobs[k].xcd_map = 0;
        const uint64_t tiles = h->info.nnz == 0 ? 0 : gl->jobs[k].ntiles;
        gl->prefix[k + 1] = gl->prefix[k] + tiles;
        gl->oprefix[k + 1] = gl->oprefix[k] + h->info.dims[modes[j]] * (uint64_t)ranks[j];
        lds = std::max(lds, lds_bytes(gl->jobs[k], threads));
    }
    gl->lds = lds;
    gl->kern = pick_kernel(g.lpn, g.fdt, g.words, gl->jobs[0].nmodes, true);
    if (gl->prefix[nj] == 0) return ALTO_OK;
    alto_status lst = check_launch_lds(gl->kern, lds, dev);
    if (lst != ALTO_OK) return lst;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, gl->kern, threads, lds) != hipSuccess || occ < 1) {
        (void)hipGetLastError();
        occ = 1;
    }
    uint64_t grid = (uint64_t)device_cus(dev) * occ;
    gl->xcd_map = 1;
    if (grid >= gl->prefix[nj]) {
        grid = gl->prefix[nj];
        gl->xcd_map = 0;
    } else {
        grid = grid / 8 * 8;
    }
    gl->grid = (unsigned)grid;
    return ALTO_OK;
}

// Per-stream device staging of job descriptors: calls on one stream reuse
// its buffer in stream order; calls on different streams never share one.
struct Staging {
    void *dev = nullptr;
    size_t bytes = 0;
};
std::mutex g_stage_mu;
std::map<std::pair<int, hipStream_t>, Staging> g_stage;

alto_status launch_group(const Group &g, const alto_handle *hs, const int *modes, const int *ranks,
                         const void *const *const *factors, float *const *outs, const BatchPlan &bp,
                         hipStream_t s, int dev) {
    GroupLaunch gl;
    alto_status st0 = plan_group(g, hs, modes, ranks, factors, outs, bp, s, dev, &gl);
    if (st0 != ALTO_OK) return st0;
    const size_t need = gl.blob_bytes();
    Staging *st;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        st = &g_stage[{dev, s}];
    }
    if (st->bytes < need) {
        if (st->dev) {
            dev_free_after(st->dev, s);
            st->dev = nullptr;
            st->bytes = 0;
        }
        if (dev_alloc(&st->dev, need) != hipSuccess) return fail(ALTO_ERR_OOM, "batch staging allocation failed");
        st->bytes = need;
    }
    std::vector<char> host(need);
    gl.write_blob(host.data());
    ALTO_HIP(hipMemcpyAsync(st->dev, host.data(), need, hipMemcpyHostToDevice, s));
    return launch_planned_group(gl, st->dev, s);
}

// Tuned launch plan per kernel-variant group and item-size class.
std::mutex g_btune_mu;
std::map<std::array<int, 6>, BatchPlan> g_btune;

// Groups of the items by kernel variant, each with its tuned (tile, table
// factor); the first sight of a group class times a few plans (launching
// them, and waiting for them, on stream s).
alto_status group_items(int count, const alto_handle *hs, const int *modes, const int *ranks, const int *fdts,
                        const void *const *const *factors, float *const *outs, hipStream_t s, int dev,
                        std::vector<std::pair<Group, BatchPlan>> *out) {
    std::map<std::array<int, 4>, Group> groups;
    for (int j = 0; j < count; j++) {
        const std::array<int, 4> key = {lpn_for(ranks[j]), fdts[j], hs[j]->info.index_words,
                                        maxo_of(hs[j]->info.nmodes)};
        Group &g = groups[key];
        g.lpn = key[0];
        g.fdt = key[1];
        g.words = key[2];
        g.maxo = key[3];
        g.items.push_back(j);
    }
    for (auto &kv : groups) {
        const Group &g = kv.second;
        uint64_t nnz = 0;
        for (int j : g.items) nnz += hs[j]->info.nnz;
        // class of the group: kernel variant and the size of an average item
        // (rounded to a factor of 4), so that a serving round with a slightly
        // different job mix reuses the plan
        const double avg = nnz > 0 ? (double)nnz / g.items.size() : 1.0;
        const int ln = (int)std::floor(std::log2(avg) / 2.0);
        const std::array<int, 6> tkey = {g.lpn, g.fdt, g.words, g.maxo, ln, 0};
        BatchPlan tuned = {0, 0, 0};
        {
            std::lock_guard<std::mutex> lk(g_btune_mu);
            auto it = g_btune.find(tkey);
            if (it != g_btune.end()) tuned = it->second;
        }
        if (tuned[0] == 0) {
            // first sight of this group class: time a few (tile, table, block) plans
            hipEvent_t e0, e1;
            ALTO_HIP(hipEventCreate(&e0));
            ALTO_HIP(hipEventCreate(&e1));
            float best = 1e30f;
            // candidates: the winners of a sweep over tile {1024, 4096} x
            // table {1/4, 1/2, 1} x threads {256, 512} on a 32-job serving
            // mix (quarter tables and full tables at 256 threads never won)
            BatchPlan bestp = {4096, 2, 256};
            for (int tile : {1024, 4096}) {
                for (const std::array<int, 2> ft : {std::array<int, 2>{2, 256}, std::array<int, 2>{2, 512},
                                                    std::array<int, 2>{4, 512}}) {
                    const int f = ft[0], th = ft[1];
                    const BatchPlan bp = {tile, f, th};
                    alto_status st = launch_group(g, hs, modes, ranks, factors, outs, bp, s, dev);
                    if (st == ALTO_ERR_ARG && th > 256) continue;  // LDS of the larger block does not fit
                    if (st != ALTO_OK) return st;
                    ALTO_HIP(hipEventRecord(e0, s));
                    st = launch_group(g, hs, modes, ranks, factors, outs, bp, s, dev);
                    if (st != ALTO_OK) return st;
                    ALTO_HIP(hipEventRecord(e1, s));
                    ALTO_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    ALTO_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best) {
                        best = ms;
                        bestp = bp;
                    }
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            tuned = bestp;
            std::lock_guard<std::mutex> lk(g_btune_mu);
            g_btune[tkey] = tuned;
        }
        out->push_back({g, tuned});
    }
    return ALTO_OK;
}

}  // namespace

alto_status batched_run(int count, const alto_handle *hs, const int *modes, const int *ranks, const int *fdts,
                        const void *const *const *factors, float *const *outs, hipStream_t s) {
    int dev = 0;
    ALTO_HIP(hipGetDevice(&dev));
    std::vector<std::pair<Group, BatchPlan>> groups;
    alto_status st = group_items(count, hs, modes, ranks, fdts, factors, outs, s, dev, &groups);
    if (st != ALTO_OK) return st;
    for (const auto &gt : groups) {
        st = launch_group(gt.first, hs, modes, ranks, factors, outs, gt.second, s, dev);
        if (st != ALTO_OK) return st;
    }
    return ALTO_OK;
}

alto_status batched_plan(int count, const alto_handle *hs, const int *modes, const int *ranks, const int *fdts,
                         const void *const *const *factors, float *const *outs, hipStream_t s,
                         std::vector<GroupLaunch> *out) {
    int dev = 0;
    ALTO_HIP(hipGetDevice(&dev));
    std::vector<std::pair<Group, BatchPlan>> groups;
    alto_status st = group_items(count, hs, modes, ranks, fdts, factors, outs, s, dev, &groups);
    if (st != ALTO_OK) return st;
    for (const auto &gt : groups) {
        GroupLaunch gl;
        st = plan_group(gt.first, hs, modes, ranks, factors, outs, gt.second, s, dev, &gl);
        if (st != ALTO_OK) return st;
        out->push_back(std::move(gl));
    }
    return ALTO_OK;
}

alto_status launch_planned_group(const GroupLaunch &gl, const void *dblob, hipStream_t s) {
    const int nj = gl.nj;
    const MttkrpArgs *djobs = (const MttkrpArgs *)dblob;
    const uint64_t *dprefix = (const uint64_t *)((const char *)dblob + gl.jobs_bytes());
    const uint64_t *doprefix = (const uint64_t *)((const char *)dblob + gl.jobs_bytes() + gl.prefix_bytes());
    {
        void *args[] = {(void *)&djobs, (void *)&doprefix, (void *)&nj};
        const unsigned g0 = grid_for(gl.oprefix[nj], 256, 8192);
        ALTO_HIP(hipLaunchKernel(zero_outputs_kernel(), dim3(g0), dim3(256), args, 0, s));
    }
    if (gl.prefix[nj] == 0) return ALTO_OK;
    int xcd_map = gl.xcd_map;
    void *args[] = {(void *)&djobs, (void *)&dprefix, (void *)&nj, (void *)&xcd_map};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = timing_begin(s, &e0, &e1);
    ALTO_HIP(hipLaunchKernel(gl.kern, dim3(gl.grid), dim3(gl.threads), args, gl.lds, s));
    if (timed) timing_end(s, e0, e1);
    return ALTO_OK;
}

}  // namespace alto

using namespace alto;

extern "C" {

// Project-written autotuner: times a small grid of launch plans around the
// default (tile length x LDS table rows, LDS-merged conflict resolution, plus
// direct atomics when fiber reuse is low) with HIP events on the caller's
// stream and keeps the fastest.  The result is recorded for the handle and
// in a process-wide cache keyed by the tensor's class, so later tensors of
// the same class skip the search.
alto_status alto_autotune(alto_handle h, int mode, int rank, alto_dtype fdt, const void *const *factors, float *out,
                          void *stream, alto_mttkrp_plan *chosen) {
    alto_status st = check_mttkrp_args(h, mode, rank, fdt, factors, out);
    if (st != ALTO_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (rank % 4 == 0) return autotune_run(h, mode, rank, fdt, factors, out, s, chosen);
    // a rank that is not a multiple of 4 is tuned (and later run) padded
    const int R4 = padded_rank(rank);
    void *pf[ALTO_MAX_MODES];
    st = pad_factors(h, rank, fdt, factors, mode, pf, s);
    if (st != ALTO_OK) return st;
    st = ensure_ws((void **)&h->ws_pad_out, &h->ws_pad_out_bytes, h->info.dims[mode] * (size_t)R4 * 4, s);
    if (st != ALTO_OK) return st;
    st = autotune_run(h, mode, R4, fdt, (const void *const *)pf, h->ws_pad_out, s, chosen);
    if (st != ALTO_OK) return st;
    launch_copy_cols(h->ws_pad_out, R4, out, rank, h->info.dims[mode], 4, s);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

}  // extern "C"

namespace alto {

// The autotuner proper, at a rank that is a multiple of 4.
alto_status autotune_run(alto_tensor *h, int mode, int rank, int fdt, const void *const *factors, float *out,
                         hipStream_t s, alto_mttkrp_plan *chosen) {
    alto_status st = ALTO_OK;
    const alto_mttkrp_plan base = default_plan(h, mode, rank, fdt);
    std::vector<alto_mttkrp_plan> cands;
    const uint64_t nnz = h->info.nnz;
    for (int threads : {256, 512}) {
        for (int tile : {2048, 4096, 8192, 16384, 32768, 65536}) {
            if (nnz > 0 && (uint64_t)tile * 64 > nnz && tile != base.tile_nnz) continue;  // keep >= 64 tiles
            for (int f : {1, 2, 4}) {
                alto_mttkrp_plan p = base;
                p.conflict = ALTO_CR_TILE;
                p.rank_tile = 0;
                p.block_threads = threads;
                p.tile_nnz = tile;
                p.table_slots = std::max(64, base.table_slots * f / 2);
                if (!tile_plan_fits(h, rank, p.table_slots, threads)) continue;
                cands.push_back(p);
            }
        }
    }
    // rank tiles for the table merge at high rank
    for (int rt : {rank / 2, rank / 4}) {
        if (rt < 8 || rt % 4 || rank % rt) continue;
        for (int tile : {4096, 16384}) {
            for (int threads : {256, 512}) {
                for (int f : {1, 2}) {
                    alto_mttkrp_plan p = base;
                    p.conflict = ALTO_CR_TILE;
                    p.tile_nnz = tile;
                    p.rank_tile = rt;
                    p.block_threads = threads;
                    p.table_slots = std::max(64, pow2_floor(8192 / rt) * f);
                    if (!tile_plan_fits(h, rt, p.table_slots, threads)) continue;
                    cands.push_back(p);
                }
            }
        }
    }
    // the whole mode in LDS, for short modes (the tile length sets only the
    // stretch granularity there: the default's and a long one)
    for (int rt = rank; rt >= 4; rt /= 2) {
        if (rt % 4 || rank % rt) break;
        for (int threads : {256, 512}) {
            if ((size_t)h->info.dims[mode] * (rt + 1) * 4 > direct_table_limit(h, threads)) continue;
            for (int tile : {base.tile_nnz, 16384}) {
                if (tile == 16384 && base.tile_nnz == 16384) continue;
                if (nnz > 0 && (uint64_t)tile * 64 > nnz && tile != base.tile_nnz) continue;
                alto_mttkrp_plan p = base;
                p.conflict = ALTO_CR_DIRECT;
                p.rank_tile = rt == rank ? 0 : rt;
                p.block_threads = threads;
                p.tile_nnz = tile;
                cands.push_back(p);
            }
        }
    }
    const double reuse = nnz / (double)h->info.dims[mode];
    if (reuse <= 8.0) {
        alto_mttkrp_plan p = base;
        p.conflict = ALTO_CR_RUN;
        cands.push_back(p);
    }
    for (auto &p : cands) accuracy_policy(h, mode, rank, &p);
    // plans the policy moved to FP64: time the other FP64 form too
    const size_t nbase = cands.size();
    for (size_t i = 0; i < nbase; i++) {
        alto_mttkrp_plan p = cands[i];
        if (alternate_f64(h, mode, rank, &p)) cands.push_back(p);
    }
    hipEvent_t e0, e1;
    ALTO_HIP(hipEventCreate(&e0));
    ALTO_HIP(hipEventCreate(&e1));
    // one warm launch, then two timed ones
    auto time_plan = [&](const alto_mttkrp_plan &p, float *ms) -> alto_status {
        alto_status r = run_mttkrp(h, mode, rank, fdt, factors, out, p, s);
        if (r != ALTO_OK) return r;
        ALTO_HIP(hipEventRecord(e0, s));
        for (int k = 0; k < 2; k++) {
            r = run_mttkrp(h, mode, rank, fdt, factors, out, p, s);
            if (r != ALTO_OK) return r;
        }
        ALTO_HIP(hipEventRecord(e1, s));
        ALTO_HIP(hipEventSynchronize(e1));
        ALTO_HIP(hipEventElapsedTime(ms, e0, e1));
        return ALTO_OK;
    };
    std::vector<std::pair<float, alto_mttkrp_plan>> timed;
    for (const auto &p : cands) {
        float ms = 0.f;
        st = time_plan(p, &ms);
        if (st != ALTO_OK) break;
        timed.push_back({ms, p});
    }
    // the three fastest again with their tiles dealt round-robin within each
    // XCD (tile order is a property of the launch, independent of the rest)
    if (st == ALTO_OK) {
        std::stable_sort(timed.begin(), timed.end(),
                         [](const std::pair<float, alto_mttkrp_plan> &x, const std::pair<float, alto_mttkrp_plan> &y) {
                             return x.first < y.first;
                         });
        const size_t top = std::min<size_t>(3, timed.size());
        for (size_t i = 0; i < top && st == ALTO_OK; i++) {
            alto_mttkrp_plan p = timed[i].second;
            if (p.conflict == ALTO_CR_HOT) continue;
            p.tile_order = ALTO_ORDER_INTERLEAVED;
            float ms = 0.f;
            st = time_plan(p, &ms);
            if (st == ALTO_OK) timed.push_back({ms, p});
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ALTO_OK) return st;
    alto_mttkrp_plan bestp = base;
    float best = 1e30f;
    for (const auto &tp : timed)
        if (tp.first < best) {
            best = tp.first;
            bestp = tp.second;
        }
    record_tuned(h, mode, rank, fdt, bestp);
    st = run_mttkrp(h, mode, rank, fdt, factors, out, bestp, s);
    if (st != ALTO_OK) return st;
    if (chosen) *chosen = bestp;
    return ALTO_OK;
}

}  // namespace alto

extern "C" {

alto_status alto_mttkrp_batched(int count, const alto_handle *hs, const int *modes, const int *ranks, const int *fdts,
                                const void *const *const *factors, float *const *outs, void *stream) {
    if (count < 0) return fail(ALTO_ERR_ARG, "count < 0");
    if (count == 0) return ALTO_OK;
    if (!hs || !modes || !ranks || !fdts || !factors || !outs) return fail(ALTO_ERR_ARG, "NULL argument");
    for (int j = 0; j < count; j++) {
        if (!factors[j]) return fail(ALTO_ERR_ARG, "factors[" + std::to_string(j) + "] is NULL");
        alto_status st = check_mttkrp_args(hs[j], modes[j], ranks[j], fdts[j], factors[j], outs[j]);
        if (st != ALTO_OK) return fail(st, "item " + std::to_string(j) + ": " + alto_last_error());
        if (ranks[j] % 4) return fail(ALTO_ERR_ARG, "item " + std::to_string(j) + ": batched ranks must be multiples of 4");
    }
    return batched_run(count, hs, modes, ranks, fdts, factors, outs, (hipStream_t)stream);
}

}  // extern "C"
