// Batched and served forms of the RASTER library.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

#include "raster.h"
#include "raster_runtime.h"

using namespace rst;

static raster_status job_scale(const raster_job& j, double* s) {
    if (j.scale > 0.0) {
        *s = j.scale;
        return RASTER_OK;
    }
    if (!scale_for_precision(j.precision, s)) return fail(RASTER_E_INVAL, "precision %d outside [0, 15]", j.precision);
    return RASTER_OK;
}

extern "C" raster_status raster_cluster_batch(const raster_job* jobs, int32_t n_jobs, hipStream_t stream,
                                              raster_result** outs) {
    if (n_jobs < 0 || (n_jobs > 0 && (!jobs || !outs))) return fail(RASTER_E_INVAL, "bad batch arguments");
    for (int32_t i = 0; i < n_jobs; ++i) outs[i] = nullptr;
    for (int32_t i = 0; i < n_jobs; ++i) {
        double s;
        raster_status st = job_scale(jobs[i], &s);
        if (st == RASTER_OK) st = raster_cluster_scaled(jobs[i].d_points, jobs[i].n, jobs[i].dt, s, jobs[i].tau,
                                                         jobs[i].mu, stream, &outs[i]);
        if (st != RASTER_OK) {
            for (int32_t k = 0; k < n_jobs; ++k) {
                raster_result_free(outs[k]);
                outs[k] = nullptr;
            }
            return st;
        }
    }
    return RASTER_OK;
}

// ---------------------------------------------------------------- server ---

struct ServerJob {
    uint64_t ticket;
    raster_job job;
    std::chrono::steady_clock::time_point submitted;
    bool done = false;
    raster_status status = RASTER_OK;
    raster_result* result = nullptr;
    double latency = 0.0;
};

struct raster_server {
    size_t budget = 0;
    int slots = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ServerJob*> queue;
    std::unordered_map<uint64_t, ServerJob*> jobs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    hipStream_t stream = nullptr;
    int device = 0;
};

static size_t job_bytes(const raster_job& j) {
    // table (16 B/slot at load 0.5 for up to n/8 tiles) + spill + outputs
    const uint64_t n = (uint64_t)std::max<int64_t>(j.n, 1);
    return (size_t)(n / 8 * 32 + n * 12 + n / 8 * 40 + (1 << 20));
}

static void server_loop(raster_server* s) {
    (void)hipSetDevice(s->device);
    while (true) {
        ServerJob* j = nullptr;
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv_work.wait(g, [&] { return s->stop || !s->queue.empty(); });
            if (s->queue.empty()) return;
            j = s->queue.front();
            s->queue.pop_front();
        }
        double sc = 0;
        raster_status st = job_scale(j->job, &sc);
        raster_result* r = nullptr;
        if (st == RASTER_OK)
            st = raster_cluster_scaled(j->job.d_points, j->job.n, j->job.dt, sc, j->job.tau, j->job.mu, s->stream, &r);
        const auto t1 = std::chrono::steady_clock::now();
        {
            std::lock_guard<std::mutex> g(s->mu);
            j->status = st;
            j->result = r;
            j->latency = std::chrono::duration<double>(t1 - j->submitted).count();
            j->done = true;
        }
        s->cv_done.notify_all();
    }
}

extern "C" raster_status raster_server_create(size_t budget_bytes, int32_t max_slots, raster_server** srv) {
    if (!srv) return fail(RASTER_E_INVAL, "srv is NULL");
    *srv = nullptr;
    if (budget_bytes == 0 || max_slots < 1) return fail(RASTER_E_INVAL, "budget and slots must be positive");
    raster_server* s = new raster_server();
    s->budget = budget_bytes;
    s->slots = max_slots;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "server stream");
    }
    s->worker = std::thread(server_loop, s);
    *srv = s;
    return RASTER_OK;
}

extern "C" raster_status raster_server_submit(raster_server* s, const raster_job* job, uint64_t* ticket) {
    if (!s || !job || !ticket) return fail(RASTER_E_INVAL, "NULL argument");
    raster_status st = check_points(job->d_points, job->n, job->dt);
    if (st != RASTER_OK) return st;
    double sc;
    st = job_scale(*job, &sc);
    if (st == RASTER_OK) st = check_params(sc, job->tau, job->mu);
    if (st != RASTER_OK) return st;
    if (job_bytes(*job) > s->budget) return fail(RASTER_E_BUDGET, "job needs more device memory than the budget");
    ServerJob* j = new ServerJob();
    j->job = *job;
    j->submitted = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> g(s->mu);
        j->ticket = s->next_ticket++;
        s->jobs[j->ticket] = j;
        s->queue.push_back(j);
    }
    s->cv_work.notify_one();
    *ticket = j->ticket;
    return RASTER_OK;
}

extern "C" raster_status raster_server_wait(raster_server* s, uint64_t ticket, raster_result** out,
                                           double* latency_s) {
    if (!s || !out) return fail(RASTER_E_INVAL, "NULL argument");
    *out = nullptr;
    ServerJob* j = nullptr;
    {
        std::unique_lock<std::mutex> g(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) return fail(RASTER_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
        j = it->second;
        s->cv_done.wait(g, [&] { return j->done; });
        s->jobs.erase(it);
    }
    raster_status st = j->status;
    *out = j->result;
    if (latency_s) *latency_s = j->latency;
    delete j;
    if (st != RASTER_OK) return fail(st, "job failed: %s", raster_status_string(st));
    return RASTER_OK;
}

extern "C" void raster_server_destroy(raster_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->jobs) {
        raster_result_free(kv.second->result);
        delete kv.second;
    }
    (void)hipStreamDestroy(s->stream);
    delete s;
}
