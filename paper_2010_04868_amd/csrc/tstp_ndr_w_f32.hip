// Weighted radius-2/3 band kernels, float.
#include "tstp_ndr_launch.hpp"

namespace tvs {
hipError_t launch_ndr_w_f32(const Problem& p, const BandGeom& g, const float* in, float* out,
                           const Coeffs<float>& cf, hipStream_t st) {
    return ndr::dispatch_w<float>(p, g, in, out, cf, st);
}
}  // namespace tvs
