// Continuous-batching request server for stencil solves.
//
// Requests (a problem, its weights, T and a host input grid) are queued on
// submit.  A worker thread repeats:
//   1. admit queued requests in arrival order while a slot is free and the
//      request's device footprint fits the remaining HBM budget (a request
//      that does not fit blocks the ones behind it, so large requests are
//      not starved); an admitted request gets a plan, a device grid and its
//      input copied in, and stays resident until it finishes;
//   2. run one chunk: every resident grid advances by min(chunk_steps,
//      remaining steps) in one batched launch set (stencil_batch_run's
//      round kernels), so requests that arrived while others were running
//      share launches with them;
//   3. retire grids that reached T: copy the result out, free the device
//      memory, timestamp, and wake waiters.
// Chunking is exact: run(T1) followed by run(T2) is bit-identical to
// run(T1+T2) for every schedule, so a served result equals the result of the
// same solve run alone.
//
// TVS_SERVER_SIMULATE=1 at create time selects a simulated executor that
// makes no device call (chunks only advance step counters and results are
// the inputs); it exists to test the scheduling policy without a GPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "api_internal.hpp"
#include "plan.hpp"

namespace tvs {
int batch_run(int n, tvs_plan* const* plans, void* const* grids, const double* const* coeffs,
              const int64_t* T, hipStream_t st, bool use_graph);
}

using namespace tvs;

namespace {

enum ReqState { QUEUED = 0, RESIDENT = 1, DONE = 2, FAILED = 3 };

struct Req {
    uint64_t id = 0;
    Problem prob;
    std::vector<double> coeffs;
    std::vector<unsigned char> host;  // input at submit, result when done
    int64_t T = 0, done = 0;
    size_t footprint = 0;
    tvs_plan* plan = nullptr;
    void* dgrid = nullptr;
    double t_arrival = 0, t_admit = 0, t_start = -1, t_finish = 0;
    int state = QUEUED;
    int error = TVS_OK;
};

}  // namespace

struct tvs_server {
    size_t budget = 0;
    int max_slots = 0;
    int chunk_steps = 0;
    bool simulate = false;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::deque<Req*> queue;
    std::vector<Req*> resident;
    std::map<uint64_t, Req*> reqs;
    uint64_t next_id = 1;
    size_t bytes_in_use = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    tvs_server_stats stats{};
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

size_t footprint_of(const Problem& p) {
    const size_t grid = p.bytes();
    return grid * (p.dependence == TVS_JACOBI ? 2 : 1) + 4096;
}

// Allocate and fill the device side of an admitted request (worker thread).
int admit_device(tvs_server* s, Req* r) {
    if (s->simulate) return TVS_OK;
    int rc = stencil_plan(&r->plan, r->prob.ndim, r->prob.dims, r->prob.dtype, r->prob.shape,
                          r->prob.order, r->prob.dependence, r->prob.boundary, nullptr);
    if (rc) return rc;
    if (hipMalloc(&r->dgrid, r->prob.bytes()) != hipSuccess)
        return set_error(TVS_E_NOMEM, "request grid allocation failed");
    if (hipMemcpyAsync(r->dgrid, r->host.data(), r->prob.bytes(), hipMemcpyHostToDevice,
                       s->stream) != hipSuccess)
        return set_error(TVS_E_DEVICE, "request upload failed");
    return ensure_scratch(r->plan);
}

void release_device(Req* r) {
    if (r->dgrid) (void)hipFree(r->dgrid);
    r->dgrid = nullptr;
    if (r->plan) stencil_plan_destroy(r->plan);
    r->plan = nullptr;
}

void worker_loop(tvs_server* s) {
    if (!s->simulate) (void)hipSetDevice(s->device);
    for (;;) {
        std::vector<Req*> chunk;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->resident.empty(); });
            if (s->stop) return;
            // 1. admission, in arrival order
            while (!s->queue.empty() && (int)s->resident.size() < s->max_slots &&
                   s->bytes_in_use + s->queue.front()->footprint <= s->budget) {
                Req* r = s->queue.front();
                s->queue.pop_front();
                s->bytes_in_use += r->footprint;
                r->t_admit = s->now();
                r->state = RESIDENT;
                s->resident.push_back(r);
                s->stats.admitted++;
            }
            chunk = s->resident;
            s->stats.resident = s->resident.size();
            s->stats.bytes_in_use = s->bytes_in_use;
        }
        if (chunk.empty()) continue;
        // device setup of newly admitted requests (outside the lock)
        for (Req* r : chunk)
            if (!s->simulate && !r->plan && r->error == TVS_OK) {
                int rc = admit_device(s, r);
                if (rc) r->error = rc;
            }
        // 2. one chunk for every resident grid
        std::vector<tvs_plan*> plans;
        std::vector<void*> grids;
        std::vector<const double*> coeffs;
        std::vector<int64_t> steps;
        std::vector<Req*> members;
        const double t_chunk = s->now();
        for (Req* r : chunk) {
            if (r->error) continue;
            const int64_t n = std::min<int64_t>(s->chunk_steps, r->T - r->done);
            if (r->t_start < 0) r->t_start = t_chunk;
            if (n <= 0) continue;
            members.push_back(r);
            plans.push_back(r->plan);
            grids.push_back(r->dgrid);
            coeffs.push_back(r->coeffs.data());
            steps.push_back(n);
        }
        int rc = TVS_OK;
        if (!members.empty() && !s->simulate)
            rc = batch_run((int)members.size(), plans.data(), grids.data(), coeffs.data(),
                           steps.data(), s->stream, false);
        const double t_end = s->now();
        // 3. advance, retire
        std::vector<Req*> finished;
        for (size_t i = 0; i < members.size(); ++i) {
            if (rc) members[i]->error = rc;
            else members[i]->done += steps[i];
        }
        for (Req* r : chunk)
            if (r->error || r->done >= r->T) finished.push_back(r);
        for (Req* r : finished) {
            if (!r->error && !s->simulate && r->T > 0) {
                if (hipMemcpy(r->host.data(), r->dgrid, r->prob.bytes(), hipMemcpyDeviceToHost) !=
                    hipSuccess)
                    r->error = TVS_E_DEVICE;
            }
            if (!s->simulate) release_device(r);
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stats.chunks++;
            s->stats.busy_seconds += t_end - t_chunk;
            for (size_t i = 0; i < members.size(); ++i)
                if (!rc)
                    s->stats.updates += (double)members[i]->prob.updated_points() * steps[i];
            const double tf = s->now();
            for (Req* r : finished) {
                r->t_finish = tf;
                r->state = r->error ? FAILED : DONE;
                s->bytes_in_use -= r->footprint;
                s->resident.erase(std::find(s->resident.begin(), s->resident.end(), r));
                s->stats.completed++;
            }
            s->stats.resident = s->resident.size();
            s->stats.bytes_in_use = s->bytes_in_use;
        }
        if (!finished.empty()) s->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

int stencil_server_create(tvs_server** out, size_t hbm_budget, int max_slots, int chunk_steps) {
    clear_error();
    if (!out) return set_error(TVS_E_INVALID, "out is NULL");
    if (max_slots < 0 || chunk_steps < 0) return set_error(TVS_E_INVALID, "negative limit");
    auto* s = new (std::nothrow) tvs_server();
    if (!s) return set_error(TVS_E_NOMEM, "host allocation");
    s->budget = hbm_budget ? hbm_budget : ((size_t)4 << 30);
    s->max_slots = max_slots ? max_slots : 64;
    s->chunk_steps = chunk_steps ? chunk_steps : 64;
    const char* sim = std::getenv("TVS_SERVER_SIMULATE");
    s->simulate = sim && sim[0] == '1';
    s->t0 = std::chrono::steady_clock::now();
    if (!s->simulate) {
        (void)hipGetDevice(&s->device);
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return set_error(TVS_E_DEVICE, "stream creation failed");
        }
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return TVS_OK;
}

int stencil_server_submit(tvs_server* s, const tvs_request* rq, uint64_t* id) {
    clear_error();
    if (!s || !rq || !id || !rq->coeffs || !rq->host_in)
        return set_error(TVS_E_INVALID, "NULL argument");
    if (rq->T < 0) return set_error(TVS_E_INVALID, "T < 0");
    auto* r = new Req();
    int rc = validate(&r->prob, rq->ndim, rq->dims, rq->dtype, rq->shape, rq->order,
                      rq->dependence, rq->boundary);
    if (rc) {
        delete r;
        return rc;
    }
    r->coeffs.assign(rq->coeffs, rq->coeffs + r->prob.order);
    r->host.assign((const unsigned char*)rq->host_in,
                   (const unsigned char*)rq->host_in + r->prob.bytes());
    r->T = rq->T;
    r->footprint = footprint_of(r->prob);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.submitted++;
        if (r->footprint > s->budget) {
            s->stats.rejected++;
            delete r;
            return set_error(TVS_E_BUSY, "request footprint exceeds the server's HBM budget");
        }
        r->id = s->next_id++;
        r->t_arrival = s->now();
        s->reqs[r->id] = r;
        s->queue.push_back(r);
        *id = r->id;
    }
    s->cv_work.notify_one();
    return TVS_OK;
}

static int finish_poll(tvs_server* s, Req* r, void* host_out, double* t_out) {
    if (t_out) {
        t_out[0] = r->t_arrival;
        t_out[1] = r->t_admit;
        t_out[2] = r->t_start;
        t_out[3] = r->t_finish;
    }
    const int err = r->error;
    if (host_out && !err) std::memcpy(host_out, r->host.data(), r->host.size());
    s->reqs.erase(r->id);
    delete r;
    return err ? set_error(err, "request failed") : TVS_OK;
}

int stencil_server_poll(tvs_server* s, uint64_t id, int* status, void* host_out, double* t_out) {
    clear_error();
    if (!s || !status) return set_error(TVS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return set_error(TVS_E_NOTFOUND, "unknown request id");
    Req* r = it->second;
    if (r->state != DONE && r->state != FAILED) {
        *status = 0;
        return TVS_OK;
    }
    *status = 1;
    return finish_poll(s, r, host_out, t_out);
}

int stencil_server_wait(tvs_server* s, uint64_t id, void* host_out, double* t_out) {
    clear_error();
    if (!s) return set_error(TVS_E_INVALID, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return set_error(TVS_E_NOTFOUND, "unknown request id");
    Req* r = it->second;
    s->cv_done.wait(lk, [&] { return r->state == DONE || r->state == FAILED || s->stop; });
    if (r->state != DONE && r->state != FAILED) return set_error(TVS_E_INVALID, "server stopped");
    return finish_poll(s, r, host_out, t_out);
}

int stencil_server_stats(tvs_server* s, tvs_server_stats* out) {
    clear_error();
    if (!s || !out) return set_error(TVS_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return TVS_OK;
}

double stencil_server_now(tvs_server* s) { return s ? s->now() : 0.0; }

int stencil_server_destroy(tvs_server* s) {
    clear_error();
    if (!s) return TVS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->reqs) {
        if (!s->simulate) release_device(kv.second);
        delete kv.second;
    }
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return TVS_OK;
}

}  // extern "C"
