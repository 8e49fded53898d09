// Deferred reporting of Gauss-Seidel kernel aborts (bounded waits that expired).
#include "api_internal.hpp"

namespace tvs {

int gs_check_status(tvs_plan* p, hipStream_t st) {
    if (!p->gs_status_host) {
        void* h = nullptr;
        if (hipHostMalloc(&h, sizeof(int), hipHostMallocDefault) != hipSuccess)
            return set_error(TVS_E_NOMEM, "hipHostMalloc of the status word failed");
        p->gs_status_host = (int*)h;
        *p->gs_status_host = 0;
        TVS_HIP_TRY(hipEventCreateWithFlags(&p->gs_status_event, hipEventDisableTiming));
    } else if (hipEventQuery(p->gs_status_event) == hipSuccess && *p->gs_status_host != 0) {
        return set_error(TVS_E_DEVICE, "a Gauss-Seidel launch timed out waiting for a "
                                       "dependency; results of that run are invalid");
    }
    TVS_HIP_TRY(hipMemcpyAsync(p->gs_status_host, (int*)p->gs_work + 1, sizeof(int),
                               hipMemcpyDeviceToHost, st));
    TVS_HIP_TRY(hipEventRecord(p->gs_status_event, st));
    return TVS_OK;
}

}  // namespace tvs
