// Internal plan object and helpers shared by the C-ABI translation units.
#pragma once

#include <string>
#include <vector>

#include "kernels.hpp"

// A Jacobi run as the graph replay cache identifies it.
struct RunKey {
    void* grid = nullptr;
    int64_t T = -1;
    std::vector<double> coeffs;
};
struct RunGraph {
    RunKey key;
    hipGraphExec_t exec = nullptr;
};

struct tvs_plan {
    tvs::Problem prob;
    tvs::Schedule sched;
    bool sched_given = false;  // the schedule came from a tuning string or the tuning cache
    void* scratch = nullptr;  // Jacobi second buffer
    size_t scratch_bytes = 0;
    void* gs_work = nullptr;  // Gauss-Seidel ticket, status word, progress counters
    size_t gs_work_bytes = 0;
    bool external_scratch = false;  // scratch/gs_work lent by the owner (server arena)
    RunKey last_run;                   // the previous eager run (graph replay cache)
    std::vector<RunGraph> run_graphs;  // captured repeated runs
    hipStream_t capture_stream = nullptr;
    int* gs_status_host = nullptr;  // pinned copy of the status word
    hipEvent_t gs_status_event = nullptr;
};

namespace tvs {

// Coefficients in the plan's precision, laid out as the kernels take them.
struct CoeffBuf {
    alignas(16) unsigned char bytes[sizeof(Coeffs<double, kMaxWeights>)];
};

void fill_coeffs(const Problem& p, const double* c, CoeffBuf* out);
int ensure_scratch(tvs_plan* p);
int enqueue_run(tvs_plan* p, void* grid, const double* coeffs, int64_t T, hipStream_t st);
int enqueue_jacobi(tvs_plan* p, void* grid, const CoeffBuf& cb, int64_t T, hipStream_t st);
int enqueue_gs(tvs_plan* p, void* grid, const CoeffBuf& cb, int64_t T, hipStream_t st);

// Gauss-Seidel status.  gs_report_previous: TVS_E_DEVICE (and the word
// cleared) if the copy queued after an earlier run has arrived and shows an
// abort.  gs_queue_status_copy: queue a copy of the status word after the run
// just enqueued on st.  gs_sync_status: wait for the plan's last copy, read
// the word itself and report (and clear) an abort.
int gs_report_previous(tvs_plan* p);
int gs_queue_status_copy(tvs_plan* p, hipStream_t st);
int gs_sync_status(tvs_plan* p);

// Autotuning cache (TVS_TUNE_CACHE): schedule for a problem, if recorded.
bool tune_cache_lookup(const Problem& p, Schedule* s);
void tune_cache_store(const Problem& p, const Schedule& s);
std::string problem_key(const Problem& p);

// Graph cache of a plan (captured launch sequences).
void graph_cache_drop(tvs_plan* p);

// Replay of repeated Jacobi runs: launches a captured graph for a run seen
// before (*done = true), or leaves it to the caller (*done = false).
int run_graph(tvs_plan* p, void* grid, const double* coeffs, int64_t T, hipStream_t st,
              bool* done);
void run_graphs_drop(tvs_plan* p);

// Device work-list buffer and its pinned host staging, kept by a caller that
// issues many batches (the server), so that a batch allocates nothing.
// Optionally also streams on which the Gauss-Seidel members of a batch run
// concurrently (each member's sweeps are one dependency chain that leaves
// most of the device idle), forked from and joined back to the batch stream.
struct BatchBuffers {
    void* dev = nullptr;
    void* host = nullptr;
    size_t capacity = 0;
    static constexpr int kAux = 4;
    int naux = 0;  // streams in aux (0: Gauss-Seidel members run on the batch stream)
    hipStream_t aux[kAux] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kAux] = {};
};

// Enqueue one batch (stencil_batch_run's work).  With ext the work lists go
// into ext asynchronously and nothing is waited for; otherwise they are
// allocated per call (use_graph: captured and cached per layout).
int batch_run(int n, tvs_plan* const* plans, void* const* grids, const double* const* coeffs,
              const int64_t* T, hipStream_t st, bool use_graph, BatchBuffers* ext);

}  // namespace tvs
