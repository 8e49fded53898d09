// Autotuner: search time-tile depth, tile shape and lane map
// for one problem on the device, keep the fastest, and remember it.
//
// The paper searched power-of-two block sizes by hand and notes that the
// performance is sensitive to them and that automatic tuning should be done
// separately (Section 4.1; future work in Section 6).  Here each candidate
// schedule that fits the hardware limits is timed with HIP events on a
// restored copy of the caller's grid, and its output is compared bit for bit
// with the first candidate's: every schedule must produce the same result, so
// a mismatch is a bug and aborts tuning.  The winner is written to the plan
// and, when TVS_TUNE_CACHE names a file, appended to it as one JSON line
// {"key": ..., "tuning": ...}; stencil_plan reads the same file.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "api_internal.hpp"
#include "plan.hpp"

namespace tvs {

std::string problem_key(const Problem& p) {
    std::ostringstream o;
    o << "nd" << p.ndim << ":";
    for (int a = 0; a < p.ndim; ++a) o << (a ? "x" : "") << p.dims[a];
    o << ":" << (p.rule == TVS_RULE_LIFE ? "life" : p.dtype == TVS_F64 ? "f64" : "f32") << ":"
      << (p.shape == TVS_BOX ? "box" : "star")
      << p.order << ":" << (p.dependence == TVS_JACOBI ? "jacobi" : "gs") << ":"
      << (p.boundary == TVS_PERIODIC ? "periodic" : "dirichlet");
    return o.str();
}

static std::mutex g_cache_mu;

bool tune_cache_lookup(const Problem& p, Schedule* s) {
    const char* path = std::getenv("TVS_TUNE_CACHE");
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::ifstream f(path);
    if (!f) return false;
    const std::string key = "\"key\": \"" + problem_key(p) + "\"";
    std::string line, found;
    while (std::getline(f, line))
        if (line.find(key) != std::string::npos) found = line;  // last entry wins
    if (found.empty()) return false;
    const std::string tag = "\"tuning\": \"";
    size_t a = found.find(tag);
    if (a == std::string::npos) return false;
    a += tag.size();
    size_t b = found.find('"', a);
    if (b == std::string::npos) return false;
    Schedule t = default_schedule(p);
    bool has_method = false;
    if (parse_tuning(found.substr(a, b - a).c_str(), &t, &has_method) != TVS_OK) return false;
    if (check_schedule(p, t) != TVS_OK) return false;
    *s = t;
    return true;
}

void tune_cache_store(const Problem& p, const Schedule& s) {
    const char* path = std::getenv("TVS_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    f << "{\"key\": \"" << problem_key(p) << "\", \"tuning\": \"" << format_tuning(p, s)
      << "\"}\n";
}

// Candidate schedules for a problem (all satisfy check_schedule).
std::vector<Schedule> tune_candidates(const Problem& p) {
    std::vector<Schedule> out;
    auto add = [&](Schedule s) {
        if (s.method == TVS_METHOD_TSTP && p.ndim >= 2 && p.dependence == TVS_JACOBI)
            choose_segment(p, &s);
        if (check_schedule(p, s) == TVS_OK) out.push_back(s);
        else clear_error();
    };
    Schedule base = default_schedule(p);
    add(base);
    Schedule plain;
    plain.method = TVS_METHOD_PLAIN;
    add(plain);
    if (p.dependence == TVS_GAUSS_SEIDEL) {
        const std::initializer_list<int> ks1 = {64, 256, 1024}, ks2 = {4, 8, 16, 32, 64, 128},
                                         ks3 = {16, 64, 256};
        for (int k : p.ndim == 1 ? ks1 : p.ndim == 2 ? ks2 : ks3) {
            Schedule s = base;
            s.k = k;
            s.c = 1;
            add(s);
        }
        return out;
    }
    if (p.ndim == 1) {
        for (int pl : {16, 64})
            for (int k : {16, 32, 64})
                for (int l : {64, 128, 256, 512, 1024}) {
                    if (k > pl) continue;
                    Schedule s = base;
                    s.pl = pl;
                    s.k = k;
                    s.l = l;
                    add(s);
                }
    } else if (p.ndim == 2 && p.radius > 1) {
        for (int c : {4, 8})
            for (int k : {1, 2, 3, 4, 6, 8})
                for (int w : {64, 128, 256, 512})
                    for (int lm : {0, 1}) {
                        Schedule s = base;
                        s.c = c;
                        s.k = k;
                        s.w = w;
                        s.lanemap = lm;
                        s.l = 0;
                        add(s);
                    }
    } else if (p.ndim == 2) {
        for (int c : {4, 8, 16})
            for (int k : {4, 6, 8, 12, 16})
                for (int w : {128, 256, 512})
                    for (int lm : {0, 1}) {
                        Schedule s = base;
                        s.kern = 0;
                        s.c = c;
                        s.k = k;
                        s.w = w;
                        s.lanemap = lm;
                        s.l = 0;
                        add(s);
                    }
    } else {
        const int shapes[][2] = {{32, 16}, {64, 16}, {64, 32}, {32, 32}, {128, 8}, {128, 16}};
        for (int c : {4, 8})
            for (int k : {1, 2, 3, 4})
                for (auto& wh : shapes)
                    for (int lm : {0, 1}) {
                        Schedule s = base;
                        s.c = c;
                        s.k = k;
                        s.w = wh[0];
                        s.h = wh[1];
                        s.lanemap = lm;
                        s.l = 0;
                        add(s);
                    }
    }
    // de-duplicate
    std::vector<Schedule> uniq;
    for (auto& s : out) {
        bool dup = false;
        for (auto& u : uniq) dup = dup || format_tuning(p, u) == format_tuning(p, s);
        if (!dup) uniq.push_back(s);
    }
    return uniq;
}

}  // namespace tvs

namespace {

__global__ void count_diff(const unsigned* a, const unsigned* b, int64_t n,
                           unsigned long long* out) {
    unsigned long long local = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        local += a[i] != b[i];
    if (local) atomicAdd(out, local);
}

__global__ void zero_u64(unsigned long long* p) { *p = 0; }

}  // namespace

using namespace tvs;

extern "C" int stencil_tune(tvs_plan* p, void* grid, const double* coeffs, int64_t T_probe,
                            void* stream, char* best, size_t best_len) {
    clear_error();
    if (!p || !grid) return set_error(TVS_E_INVALID, "NULL argument");
    static const double kNoWeights[kMaxWeights] = {};
    if (p->prob.rule == TVS_RULE_LIFE) coeffs = kNoWeights;  // the rule has no weights
    if (!coeffs) return set_error(TVS_E_INVALID, "NULL argument");
    if (T_probe < 1) return set_error(TVS_E_INVALID, "T_probe must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    const Problem& pr = p->prob;
    const size_t bytes = pr.bytes();
    std::vector<Schedule> cands = tune_candidates(pr);
    if (cands.empty()) return set_error(TVS_E_UNSUPPORTED, "no candidate schedule");
    void *saved = nullptr, *ref = nullptr;
    unsigned long long* dcount = nullptr;
    auto cleanup = [&]() {
        if (saved) (void)hipFree(saved);
        if (ref) (void)hipFree(ref);
        if (dcount) (void)hipFree(dcount);
    };
    if (hipMalloc(&saved, bytes) != hipSuccess || hipMalloc(&ref, bytes) != hipSuccess ||
        hipMalloc((void**)&dcount, sizeof(unsigned long long)) != hipSuccess) {
        cleanup();
        return set_error(TVS_E_NOMEM, "tuning buffers");
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int rc = TVS_OK;
    if (hipMemcpyAsync(saved, grid, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        rc = set_error(TVS_E_DEVICE, "saving the grid failed");
    }
    const Schedule original = p->sched;
    // bring the device to its working clocks before the first candidate is timed
    for (int w = 0; w < 4 && rc == TVS_OK; ++w) rc = enqueue_run(p, grid, coeffs, T_probe, st);
    (void)hipStreamSynchronize(st);
    double best_ms = 1e300;
    Schedule best_s = original;
    const int64_t words = (int64_t)(bytes / 4);  // every grid is whole 4-byte elements
    for (size_t i = 0; i < cands.size() && rc == TVS_OK; ++i) {
        p->sched = cands[i];
        // restore, run once (also warms up), compare with the first candidate
        (void)hipMemcpyAsync(grid, saved, bytes, hipMemcpyDeviceToDevice, st);
        rc = enqueue_run(p, grid, coeffs, T_probe, st);
        if (rc) break;
        if (i == 0) {
            (void)hipMemcpyAsync(ref, grid, bytes, hipMemcpyDeviceToDevice, st);
        } else {
            hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, st, dcount);
            hipLaunchKernelGGL(count_diff, dim3(1024), dim3(256), 0, st,
                               (const unsigned*)grid, (const unsigned*)ref,
                               words, dcount);
            unsigned long long diff = 0;
            (void)hipMemcpyAsync(&diff, dcount, sizeof diff, hipMemcpyDeviceToHost, st);
            (void)hipStreamSynchronize(st);
            if (diff) {
                rc = set_error(TVS_E_DEVICE, "schedule " + format_tuning(pr, cands[i]) +
                                                 " changed the result bits");
                break;
            }
        }
        // timed: restore + run, three times; keep the fastest.  The timed run
        // covers at least two full bands (k is capped by T, so a shorter probe
        // would time a deep schedule as a shallow one), and candidates are
        // compared per step, reported scaled to T_probe steps.
        const int64_t kc = cands[i].method == TVS_METHOD_PLAIN ? 1 : std::max(1, cands[i].k);
        const int64_t T_time = std::max<int64_t>(T_probe, 2 * kc);
        double ms_best = 1e300;
        for (int r = 0; r < 3; ++r) {
            (void)hipMemcpyAsync(grid, saved, bytes, hipMemcpyDeviceToDevice, st);
            (void)hipEventRecord(e0, st);
            rc = enqueue_run(p, grid, coeffs, T_time, st);
            (void)hipEventRecord(e1, st);
            if (rc) break;
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms_best = std::min(ms_best, (double)ms * (double)T_probe / (double)T_time);
        }
        // a Gauss-Seidel candidate whose bounded waits expired produced no result
        if (rc == TVS_OK && pr.dependence == TVS_GAUSS_SEIDEL) rc = gs_sync_status(p);
        if (rc) break;
        if (std::getenv("TVS_LOG"))
            std::fprintf(stderr, "[tvs tune] %s: %.4f ms\n", format_tuning(pr, cands[i]).c_str(),
                         ms_best);
        if (ms_best < best_ms) {
            best_ms = ms_best;
            best_s = cands[i];
        }
    }
    (void)hipMemcpyAsync(grid, saved, bytes, hipMemcpyDeviceToDevice, st);
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cleanup();
    if (rc) {
        p->sched = original;
        return rc;
    }
    p->sched = best_s;
    graph_cache_drop(p);
    run_graphs_drop(p);
    tune_cache_store(pr, best_s);
    if (best && best_len) {
        std::string t = format_tuning(pr, best_s);
        std::snprintf(best, best_len, "%s", t.c_str());
    }
    return TVS_OK;
}
