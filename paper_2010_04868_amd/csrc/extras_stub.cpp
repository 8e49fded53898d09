// Temporary: batch, tuning and serving entry points until their own units land.
#include "api_internal.hpp"
#include "plan.hpp"

namespace tvs {
bool tune_cache_lookup(const Problem&, Schedule*) { return false; }
void tune_cache_store(const Problem&, const Schedule&) {}
}  // namespace tvs

using namespace tvs;
extern "C" {
int stencil_tune(tvs_plan*, void*, const double*, int64_t, void*, char*, size_t) {
    return set_error(TVS_E_UNSUPPORTED, "not built yet");
}
int stencil_server_create(tvs_server**, size_t, int, int) { return set_error(TVS_E_UNSUPPORTED, "not built yet"); }
int stencil_server_submit(tvs_server*, const tvs_request*, uint64_t*) { return TVS_E_UNSUPPORTED; }
int stencil_server_poll(tvs_server*, uint64_t, int*, void*, double*) { return TVS_E_UNSUPPORTED; }
int stencil_server_wait(tvs_server*, uint64_t, void*, double*) { return TVS_E_UNSUPPORTED; }
int stencil_server_stats(tvs_server*, tvs_server_stats*) { return TVS_E_UNSUPPORTED; }
double stencil_server_now(tvs_server*) { return 0.0; }
int stencil_server_destroy(tvs_server*) { return TVS_E_UNSUPPORTED; }
}
