// Continuous-batching CP-ALS server: a native scheduler thread that admits
// jobs by HBM footprint, keeps their ALTO tensors resident and interleaves
// their sweeps in rounds (one batched sweep of every active job per round),
// building newly admitted tensors on a second stream while a round runs.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "alto_internal.h"
#include "memory.h"
#include "mttkrp.h"

namespace alto {
namespace {

constexpr uint32_t kServerMagic = 0x5E77E700u;

struct Job {
    alto_serve_job spec;
    uint64_t footprint = 0;
    alto_handle h = nullptr;
    int sweeps_done = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    double ms_sum = 0, ms_max = 0;
    int status = ALTO_OK;
};

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

uint64_t footprint_of(const alto_serve_job &j) {
    alto_info_t info;
    if (make_plan(j.nmodes, j.dims, &info, nullptr) != ALTO_OK) return ~uint64_t(0);
    const uint64_t words = info.index_words;
    const uint64_t tensor = j.nnz * (8 * words + 4);
    const uint64_t scratch = tensor + (j.nnz / 2048 + 1) * 256 * 12;  // build: alternate buffers + digit counts
    uint64_t factors = 0, maxI = 0;
    for (int m = 0; m < j.nmodes; m++) {
        factors += j.dims[m] * (uint64_t)j.rank * (j.fdt == ALTO_BF16 ? 6 : 4);
        maxI = std::max<uint64_t>(maxI, j.dims[m]);
    }
    uint64_t ws = maxI * j.rank * 4 + (uint64_t)(j.nmodes + 2 + 512) * j.rank * j.rank * 8 + 256;
    // a job that runs its own MTTKRP launches may accumulate in FP64
    if (j.nnz >= kBatchAloneNnz) ws += maxI * j.rank * 8;
    const uint64_t g = 2 << 20;  // allocation granule of the caching allocator, per buffer
    return tensor + scratch + factors + ws + 8 * g;
}

}  // namespace
}  // namespace alto

struct alto_server {
    uint32_t magic = alto::kServerMagic;
    int device = 0;
    uint64_t budget = 0, in_use = 0, peak = 0;
    int max_active = 1;
    std::mutex mu;
    std::condition_variable cv, drained;
    std::deque<alto::Job *> queue;
    std::vector<alto::Job *> active;
    std::deque<alto_serve_done> done;
    std::vector<double> sweep_ms;
    alto_serve_stats st{};
    bool stop = false;
    uint64_t outstanding = 0;  // submitted, not yet completed or rejected
    hipStream_t compute = nullptr, build = nullptr;
    std::thread worker;
};

namespace alto {
namespace {

void finish(alto_server *S, Job *j, int status) {
    j->status = status;
    j->t_done = now_s();
    alto_serve_done d;
    memset(&d, 0, sizeof(d));
    d.user_tag = j->spec.user_tag;
    d.status = status;
    d.sweeps = j->sweeps_done;
    d.submit_s = j->t_submit;
    d.admit_s = j->t_admit;
    d.done_s = j->t_done;
    d.sweep_ms_sum = j->ms_sum;
    d.sweep_ms_max = j->ms_max;
    S->done.push_back(d);
    S->outstanding--;
    delete j;
}

void worker_loop(alto_server *S) {
    (void)hipSetDevice(S->device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    for (;;) {
        std::vector<Job *> admit;
        std::vector<Job *> round;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->queue.empty() && S->active.empty()) {
                S->drained.notify_all();
                if (S->stop) break;
                S->cv.wait_for(lk, std::chrono::milliseconds(50));
                continue;
            }
            // first-fit admission in arrival order: a job that does not fit
            // now does not hold back smaller ones behind it
            for (auto it = S->queue.begin(); it != S->queue.end();) {
                Job *j = *it;
                if (j->footprint > S->budget) {
                    it = S->queue.erase(it);
                    S->st.rejected++;
                    S->st.queued = S->queue.size();
                    finish(S, j, ALTO_ERR_BUDGET);
                    continue;
                }
                if ((int)(S->active.size() + admit.size()) < S->max_active && S->in_use + j->footprint <= S->budget) {
                    S->in_use += j->footprint;
                    S->peak = std::max(S->peak, S->in_use);
                    admit.push_back(j);
                    it = S->queue.erase(it);
                } else {
                    ++it;
                }
            }
            S->st.queued = S->queue.size();
            round = S->active;
        }
        // launch one round (asynchronously) for the jobs already resident
        bool launched = false;
        if (!round.empty()) {
            std::vector<alto_handle> hs;
            std::vector<int> ranks, fdts;
            std::vector<float *const *> facs;
            std::vector<double *> lams;
            for (Job *j : round) {
                hs.push_back(j->h);
                ranks.push_back(j->spec.rank);
                fdts.push_back(j->spec.fdt);
                facs.push_back(j->spec.factors);
                lams.push_back(j->spec.lambda_out);
            }
            (void)hipEventRecord(e0, S->compute);
            alto_status st = cpd_als_sweep_batched((int)hs.size(), hs.data(), ranks.data(), fdts.data(),
                                                   facs.data(), lams.data(), S->compute);
            (void)hipEventRecord(e1, S->compute);
            if (st != ALTO_OK) {
                std::lock_guard<std::mutex> lk(S->mu);
                (void)hipStreamSynchronize(S->compute);
                for (Job *j : round) {
                    S->active.erase(std::find(S->active.begin(), S->active.end(), j));
                    alto_free(j->h);
                    S->in_use -= j->footprint;
                    S->st.completed++;
                    finish(S, j, st);
                }
                S->st.active = S->active.size();
                round.clear();
            } else {
                launched = true;
            }
        }
        // meanwhile, build the newly admitted tensors on the build stream
        for (Job *j : admit) {
            alto_handle h = nullptr;
            alto_status st = alto_build(j->spec.nmodes, j->spec.dims, j->spec.nnz, j->spec.coords, j->spec.vals,
                                        (void *)S->build, &h);
            std::lock_guard<std::mutex> lk(S->mu);
            S->st.admitted++;
            j->t_admit = now_s();
            if (st != ALTO_OK) {
                S->in_use -= j->footprint;
                S->st.completed++;
                finish(S, j, st);
                continue;
            }
            j->h = h;
            S->active.push_back(j);
            S->st.active = S->active.size();
        }
        if (launched) {
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            std::lock_guard<std::mutex> lk(S->mu);
            S->st.rounds++;
            for (Job *j : round) {
                j->sweeps_done++;
                j->ms_sum += ms;
                j->ms_max = std::max(j->ms_max, (double)ms);
                S->sweep_ms.push_back(ms);
                S->st.sweeps_done++;
                S->st.nnz_modes_done += j->spec.nnz * (uint64_t)j->spec.nmodes;
                if (j->sweeps_done >= j->spec.sweeps) {
                    S->active.erase(std::find(S->active.begin(), S->active.end(), j));
                    alto_free(j->h);
                    j->h = nullptr;
                    S->in_use -= j->footprint;
                    S->st.completed++;
                    finish(S, j, ALTO_OK);
                }
            }
            S->st.active = S->active.size();
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

}  // namespace
}  // namespace alto

using namespace alto;

#define ALTO_CHECK_SERVER(s)                                                                            \
    do {                                                                                                \
        if (!(s) || (s)->magic != kServerMagic) return fail(ALTO_ERR_STATE, "invalid alto server");      \
    } while (0)

extern "C" {

alto_status alto_serve_footprint(const alto_serve_job *job, uint64_t *bytes) {
    if (!job || !bytes) return fail(ALTO_ERR_ARG, "NULL argument");
    alto_info_t info;
    alto_status st = make_plan(job->nmodes, job->dims, &info, nullptr);
    if (st != ALTO_OK) return st;
    *bytes = footprint_of(*job);
    return ALTO_OK;
}

alto_status alto_server_create(uint64_t budget_bytes, int max_active, alto_server_t *out) {
    if (!out || max_active < 1 || budget_bytes == 0) return fail(ALTO_ERR_ARG, "bad server arguments");
    alto_server *S = new alto_server();
    S->budget = budget_bytes;
    S->max_active = max_active;
    if (hipGetDevice(&S->device) != hipSuccess || hipStreamCreateWithFlags(&S->compute, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&S->build, hipStreamNonBlocking) != hipSuccess) {
        delete S;
        return fail(ALTO_ERR_HIP, "server stream creation failed");
    }
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return ALTO_OK;
}

alto_status alto_server_submit(alto_server_t S, const alto_serve_job *job) {
    ALTO_CHECK_SERVER(S);
    if (!job) return fail(ALTO_ERR_ARG, "job is NULL");
    alto_info_t info;
    alto_status st = make_plan(job->nmodes, job->dims, &info, nullptr);
    if (st != ALTO_OK) return st;
    if (job->rank < 4 || job->rank > 64 || job->rank % 4 || job->sweeps < 1 ||
        (job->fdt != ALTO_F32 && job->fdt != ALTO_BF16) || !job->lambda_out)
        return fail(ALTO_ERR_ARG, "bad job (rank 4..64 multiple of 4, sweeps >= 1, dtype, lambda_out)");
    for (int m = 0; m < job->nmodes; m++)
        if (!job->factors[m] || (job->nnz && !job->coords[m])) return fail(ALTO_ERR_ARG, "NULL job pointer");
    if (job->nnz && !job->vals) return fail(ALTO_ERR_ARG, "NULL job values");
    Job *j = new Job();
    j->spec = *job;
    j->footprint = footprint_of(*job);
    j->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->queue.push_back(j);
        S->st.submitted++;
        S->st.queued = S->queue.size();
        S->outstanding++;
    }
    S->cv.notify_all();
    return ALTO_OK;
}

alto_status alto_server_poll(alto_server_t S, alto_serve_done *out, int max, int *n) {
    ALTO_CHECK_SERVER(S);
    if (!n || (max > 0 && !out)) return fail(ALTO_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    int k = 0;
    while (k < max && !S->done.empty()) {
        out[k++] = S->done.front();
        S->done.pop_front();
    }
    *n = k;
    return ALTO_OK;
}

alto_status alto_server_stats(alto_server_t S, alto_serve_stats *out) {
    ALTO_CHECK_SERVER(S);
    if (!out) return fail(ALTO_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->bytes_in_use = S->in_use;
    out->bytes_peak = S->peak;
    return ALTO_OK;
}

alto_status alto_server_drain(alto_server_t S) {
    ALTO_CHECK_SERVER(S);
    std::unique_lock<std::mutex> lk(S->mu);
    while (S->outstanding > 0) {
        S->cv.notify_all();
        S->drained.wait_for(lk, std::chrono::milliseconds(20));
    }
    return ALTO_OK;
}

alto_status alto_server_sweep_latencies(alto_server_t S, double *out, uint64_t max, uint64_t *n) {
    ALTO_CHECK_SERVER(S);
    if (!n || (max > 0 && !out)) return fail(ALTO_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    const uint64_t k = std::min<uint64_t>(max, S->sweep_ms.size());
    for (uint64_t i = 0; i < k; i++) out[i] = S->sweep_ms[i];
    *n = k;
    return ALTO_OK;
}

alto_status alto_server_destroy(alto_server_t S) {
    ALTO_CHECK_SERVER(S);
    alto_server_drain(S);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    S->worker.join();
    (void)hipStreamDestroy(S->compute);
    (void)hipStreamDestroy(S->build);
    S->magic = 0;
    delete S;
    return ALTO_OK;
}

}  // extern "C"
