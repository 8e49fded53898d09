// Continuous-batching request server for stencil solves.
//
// Requests (a problem, its weights, T and a host input grid) are queued on
// submit.  A worker thread runs a pipeline:
//   1. admission, in arrival order, while a slot is free and the request's
//      device footprint (grid, plus the Jacobi second buffer or the
//      Gauss-Seidel work area) fits in the server's device arena -- one
//      allocation of the HBM budget made at create and carved first-fit, so
//      admitting and retiring a request allocates nothing on the device.  A
//      request that does not fit blocks the ones behind it, so large requests
//      are not starved.  The input is copied in on the server's stream, ahead
//      of the request's first chunk;
//   2. one chunk: every resident grid that still has steps advances by
//      min(chunk_steps, remaining) in one batched launch set (the band-round
//      kernels of stencil_batch_run), so requests that arrived while others
//      were running share launches with them.  The chunk's work lists go into
//      one of two persistent buffers and are uploaded asynchronously;
//   3. retirement of the grids that finished in the PREVIOUS chunk: wait for
//      that chunk (the chunk just enqueued keeps the device busy meanwhile),
//      copy the results out, return their arena space, wake the waiters.
// Chunking is exact: run(T1) followed by run(T2) is bit-identical to
// run(T1+T2) for every schedule, so a served result equals the result of the
// same solve run alone.
//
// TVS_SERVER_SIMULATE=1 at create time selects a simulated executor that
// makes no device call (chunks only advance step counters and results are
// the inputs); it exists to test the scheduling policy without a GPU.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "api_internal.hpp"
#include "plan.hpp"

using namespace tvs;

namespace {

enum ReqState { QUEUED = 0, RESIDENT = 1, DONE = 2, FAILED = 3 };

constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }

struct Req {
    uint64_t id = 0;
    Problem prob;
    std::vector<double> coeffs;
    std::vector<unsigned char> host;  // input at submit, result when done
    int64_t T = 0, issued = 0;        // steps enqueued so far
    size_t footprint = 0, grid_bytes = 0, aux_bytes = 0;
    size_t arena_off = 0;
    tvs_plan* plan = nullptr;
    void* dgrid = nullptr;
    double t_arrival = 0, t_admit = 0, t_start = -1, t_finish = 0;
    int state = QUEUED;
    bool retiring = false;  // all steps enqueued; retired after its last chunk
    int error = TVS_OK;
};

// First-fit allocator over one device allocation (offsets only; the host
// never touches the memory).
class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {  // merge with the next block
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {  // merge with the previous block
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
};

// One chunk in flight: its members, the requests it finishes, timing events
// and the work-list buffers its launches read.
struct Chunk {
    std::vector<Req*> finishing;
    std::vector<std::pair<Req*, int64_t>> members;  // (request, steps)
    hipEvent_t start = nullptr, end = nullptr;
    BatchBuffers buffers;
    bool in_flight = false;
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
    Arena arena;
    char* arena_base = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    Chunk chunks[2];  // worker thread only
    std::chrono::steady_clock::time_point t0;
    tvs_server_stats stats{};
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Plan and device bytes of a request (host only).
int size_request(Req* r) {
    int rc = stencil_plan(&r->plan, r->prob.ndim, r->prob.dims, r->prob.dtype, r->prob.shape,
                          r->prob.order, r->prob.dependence, r->prob.boundary, nullptr);
    if (rc) return rc;
    r->plan->external_scratch = true;
    r->grid_bytes = align_up(r->prob.bytes());
    r->aux_bytes = r->prob.dependence == TVS_JACOBI
                       ? align_up(r->prob.bytes())
                       : align_up(gs_work_bytes(r->prob));
    r->footprint = r->grid_bytes + r->aux_bytes;
    return TVS_OK;
}

// Point the request's grid and plan scratch into its arena block and queue
// the input upload (worker thread, server stream).
int place_device(tvs_server* s, Req* r) {
    if (s->simulate) return TVS_OK;
    char* base = s->arena_base + r->arena_off;
    r->dgrid = base;
    if (r->prob.dependence == TVS_JACOBI) {
        r->plan->scratch = base + r->grid_bytes;
        r->plan->scratch_bytes = r->aux_bytes;
    } else {
        r->plan->gs_work = base + r->grid_bytes;
        r->plan->gs_work_bytes = r->aux_bytes;
        // the status word must start clear (each launch resets the rest)
        if (hipMemsetAsync(r->plan->gs_work, 0, gs_state_bytes(r->prob), s->stream) != hipSuccess)
            return set_error(TVS_E_DEVICE, "clearing the Gauss-Seidel work area failed");
    }
    if (hipMemcpyAsync(r->dgrid, r->host.data(), r->prob.bytes(), hipMemcpyHostToDevice,
                       s->stream) != hipSuccess)
        return set_error(TVS_E_DEVICE, "request upload failed");
    return TVS_OK;
}

// Copy the results of finished requests out and release their device side
// (worker thread; the chunk that finished them has completed).
void retire(tvs_server* s, const std::vector<Req*>& done) {
    for (Req* r : done) {
        if (r->error || s->simulate || r->T == 0) continue;
        if (hipMemcpy(r->host.data(), r->dgrid, r->prob.bytes(), hipMemcpyDeviceToHost) !=
            hipSuccess)
            r->error = TVS_E_DEVICE;
        // a Gauss-Seidel launch whose bounded dependency wait expired leaves a
        // non-zero status word; its result is invalid
        int status = 0;
        if (!r->error && r->prob.dependence == TVS_GAUSS_SEIDEL &&
            (hipMemcpy(&status, (const int*)r->plan->gs_work + 1, sizeof status,
                       hipMemcpyDeviceToHost) != hipSuccess ||
             status != 0))
            r->error = TVS_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    const double tf = s->now();
    for (Req* r : done) {
        if (r->plan) stencil_plan_destroy(r->plan);  // its scratch is the arena's
        r->plan = nullptr;
        r->dgrid = nullptr;
        s->arena.release(r->arena_off, r->footprint);
        s->bytes_in_use -= r->footprint;
        r->t_finish = tf;
        r->state = r->error ? FAILED : DONE;
        s->resident.erase(std::find(s->resident.begin(), s->resident.end(), r));
        s->stats.completed++;
    }
    s->stats.resident = s->resident.size();
    s->stats.bytes_in_use = s->bytes_in_use;
}

// Wait for an in-flight chunk, account for it and retire what it finished.
void complete_chunk(tvs_server* s, Chunk* c) {
    if (!c->in_flight) return;
    float ms = 0;
    if (!s->simulate) {
        if (hipEventSynchronize(c->end) != hipSuccess)
            for (auto& m : c->members) m.first->error = TVS_E_DEVICE;
        (void)hipEventElapsedTime(&ms, c->start, c->end);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.busy_seconds += ms / 1e3;
        for (auto& m : c->members)
            if (!m.first->error)
                s->stats.updates += (double)m.first->prob.updated_points() * m.second;
    }
    retire(s, c->finishing);
    c->finishing.clear();
    c->members.clear();
    c->in_flight = false;
    s->cv_done.notify_all();
}

void worker_loop(tvs_server* s) {
    if (!s->simulate) (void)hipSetDevice(s->device);
    int cur = 0;
    for (;;) {
        std::vector<Req*> admitted, active;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                return s->stop || !s->queue.empty() || !s->resident.empty() ||
                       s->chunks[0].in_flight || s->chunks[1].in_flight;
            });
            if (s->stop) return;
            // 1. admission, in arrival order
            while (!s->queue.empty() && (int)s->resident.size() < s->max_slots) {
                Req* r = s->queue.front();
                if (!s->arena.alloc(r->footprint, &r->arena_off)) break;
                s->queue.pop_front();
                s->bytes_in_use += r->footprint;
                r->t_admit = s->now();
                r->state = RESIDENT;
                s->resident.push_back(r);
                s->stats.admitted++;
                admitted.push_back(r);
            }
            for (Req* r : s->resident)
                if (!r->retiring) active.push_back(r);
            s->stats.resident = s->resident.size();
            s->stats.bytes_in_use = s->bytes_in_use;
        }
        for (Req* r : admitted) {
            int rc = place_device(s, r);
            if (rc) r->error = rc;
        }
        // 2. one chunk over the active grids; its buffers were last used by
        //    the chunk two rounds ago, which must have completed
        Chunk& c = s->chunks[cur];
        complete_chunk(s, &c);
        std::vector<tvs_plan*> plans;
        std::vector<void*> grids;
        std::vector<const double*> coeffs;
        std::vector<int64_t> steps;
        const double t_chunk = s->now();
        for (Req* r : active) {
            const int64_t n =
                r->error ? 0 : std::min<int64_t>(s->chunk_steps, r->T - r->issued);
            if (r->t_start < 0) r->t_start = t_chunk;
            if (n > 0) {
                c.members.emplace_back(r, n);
                plans.push_back(r->plan);
                grids.push_back(r->dgrid);
                coeffs.push_back(r->coeffs.data());
                steps.push_back(n);
            }
            r->issued += n;
            if (r->error || r->issued >= r->T) {
                r->retiring = true;
                c.finishing.push_back(r);
            }
        }
        const bool launched = !c.members.empty() || !c.finishing.empty();
        if (launched) {
            int rc = TVS_OK;
            if (!s->simulate) {
                (void)hipEventRecord(c.start, s->stream);
                if (!plans.empty())
                    rc = batch_run((int)plans.size(), plans.data(), grids.data(), coeffs.data(),
                                   steps.data(), s->stream, false, &c.buffers);
                (void)hipEventRecord(c.end, s->stream);
            }
            if (rc)
                for (auto& m : c.members) m.first->error = rc;
            c.in_flight = true;
            std::lock_guard<std::mutex> lk(s->mu);
            s->stats.chunks++;
        }
        // 3. retire what the previous chunk finished while this one runs
        cur ^= 1;
        complete_chunk(s, &s->chunks[cur]);
        // nothing left to overlap with: finish this chunk too
        if (launched && active.size() == c.finishing.size()) complete_chunk(s, &c);
    }
}

void destroy_chunks(tvs_server* s) {
    for (auto& c : s->chunks) {
        if (c.start) (void)hipEventDestroy(c.start);
        if (c.end) (void)hipEventDestroy(c.end);
        BatchBuffers& b = c.buffers;
        if (b.dev) (void)hipFree(b.dev);
        if (b.host) (void)hipHostFree(b.host);
        if (b.fork) (void)hipEventDestroy(b.fork);
        for (int a = 0; a < BatchBuffers::kAux; ++a) {
            if (b.aux[a]) (void)hipStreamDestroy(b.aux[a]);
            if (b.join[a]) (void)hipEventDestroy(b.join[a]);
        }
        c = Chunk();
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
    s->budget = align_up(hbm_budget ? hbm_budget : ((size_t)4 << 30));
    s->max_slots = max_slots ? max_slots : 64;
    s->chunk_steps = chunk_steps ? chunk_steps : 64;
    const char* sim = std::getenv("TVS_SERVER_SIMULATE");
    s->simulate = sim && sim[0] == '1';
    s->t0 = std::chrono::steady_clock::now();
    s->arena.reset(s->budget);
    if (!s->simulate) {
        (void)hipGetDevice(&s->device);
        int rc = TVS_OK;
        if (hipMalloc((void**)&s->arena_base, s->budget) != hipSuccess) {
            s->arena_base = nullptr;
            rc = set_error(TVS_E_NOMEM, "the server's device arena (hbm_budget) is not available");
        } else if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            s->stream = nullptr;
            rc = set_error(TVS_E_DEVICE, "stream creation failed");
        }
        for (auto& c : s->chunks) {
            if (!rc && (hipEventCreate(&c.start) != hipSuccess ||
                        hipEventCreate(&c.end) != hipSuccess))
                rc = set_error(TVS_E_DEVICE, "event creation failed");
            // Gauss-Seidel requests of a chunk run side by side on these
            // (default-priority) streams
            BatchBuffers& b = c.buffers;
            if (!rc && hipEventCreateWithFlags(&b.fork, hipEventDisableTiming) != hipSuccess)
                rc = set_error(TVS_E_DEVICE, "event creation failed");
            for (int a = 0; a < BatchBuffers::kAux && !rc; ++a) {
                if (hipStreamCreateWithFlags(&b.aux[a], hipStreamNonBlocking) != hipSuccess ||
                    hipEventCreateWithFlags(&b.join[a], hipEventDisableTiming) != hipSuccess)
                    rc = set_error(TVS_E_DEVICE, "stream creation failed");
                else
                    b.naux = a + 1;
            }
        }
        if (rc) {
            destroy_chunks(s);
            if (s->stream) (void)hipStreamDestroy(s->stream);
            if (s->arena_base) (void)hipFree(s->arena_base);
            delete s;
            return rc;
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
    if (rc == TVS_OK && r->prob.radius > 1)
        rc = set_error(TVS_E_UNSUPPORTED, "the server takes radius-1 stencils");
    if (rc == TVS_OK) rc = size_request(r);
    if (rc) {
        if (r->plan) stencil_plan_destroy(r->plan);
        delete r;
        return rc;
    }
    r->coeffs.assign(rq->coeffs, rq->coeffs + r->prob.order);
    r->host.assign((const unsigned char*)rq->host_in,
                   (const unsigned char*)rq->host_in + r->prob.bytes());
    r->T = rq->T;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.submitted++;
        if (r->footprint > s->budget) {
            s->stats.rejected++;
            stencil_plan_destroy(r->plan);
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
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->reqs) {
        if (kv.second->plan) stencil_plan_destroy(kv.second->plan);
        delete kv.second;
    }
    if (!s->simulate) {
        destroy_chunks(s);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        if (s->arena_base) (void)hipFree(s->arena_base);
    }
    delete s;
    return TVS_OK;
}

}  // extern "C"
