// Reporting of Gauss-Seidel kernel aborts.  A Gauss-Seidel launch waits for
// its producers with bounded spins; when a wait expires the kernel sets the
// status word in the plan's work area and every later wait of the plan gives
// up at once, so the results of that run and of every run after it are
// invalid until the abort has been reported.  Reporting clears the word.
#include "api_internal.hpp"

namespace tvs {

namespace {

int report_abort(tvs_plan* p) {
    const int zero = 0;
    if (p->gs_status_host) *p->gs_status_host = 0;
    // synchronous: the word is clear before any later run is enqueued
    (void)hipMemcpy((int*)p->gs_work + 1, &zero, sizeof zero, hipMemcpyHostToDevice);
    return set_error(TVS_E_DEVICE, "a Gauss-Seidel launch timed out waiting for a dependency; "
                                   "the results of the plan's runs since the last report are "
                                   "invalid");
}

}  // namespace

int gs_report_previous(tvs_plan* p) {
    if (!p->gs_status_event) return TVS_OK;
    if (hipEventQuery(p->gs_status_event) == hipSuccess && *p->gs_status_host != 0)
        return report_abort(p);
    return TVS_OK;
}

int gs_queue_status_copy(tvs_plan* p, hipStream_t st) {
    if (!p->gs_status_host) {
        void* h = nullptr;
        if (hipHostMalloc(&h, sizeof(int), hipHostMallocDefault) != hipSuccess)
            return set_error(TVS_E_NOMEM, "hipHostMalloc of the status word failed");
        p->gs_status_host = (int*)h;
        *p->gs_status_host = 0;
        TVS_HIP_TRY(hipEventCreateWithFlags(&p->gs_status_event, hipEventDisableTiming));
    }
    TVS_HIP_TRY(hipMemcpyAsync(p->gs_status_host, (int*)p->gs_work + 1, sizeof(int),
                               hipMemcpyDeviceToHost, st));
    TVS_HIP_TRY(hipEventRecord(p->gs_status_event, st));
    return TVS_OK;
}

int gs_sync_status(tvs_plan* p) {
    if (p->prob.dependence != TVS_GAUSS_SEIDEL || !p->gs_work) return TVS_OK;
    if (p->gs_status_event) TVS_HIP_TRY(hipEventSynchronize(p->gs_status_event));
    int word = 0;
    TVS_HIP_TRY(hipMemcpy(&word, (const int*)p->gs_work + 1, sizeof word, hipMemcpyDeviceToHost));
    if (word != 0) return report_abort(p);
    if (p->gs_status_host) *p->gs_status_host = 0;
    return TVS_OK;
}

}  // namespace tvs

extern "C" int stencil_plan_check(tvs_plan* plan) {
    tvs::clear_error();
    if (!plan) return tvs::set_error(TVS_E_INVALID, "NULL argument");
    return tvs::gs_sync_status(plan);
}
