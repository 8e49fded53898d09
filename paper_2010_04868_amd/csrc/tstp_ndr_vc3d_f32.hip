// Variable-coefficient 3D band kernels, float.
#include "tstp_ndr_launch.hpp"

namespace tvs {
hipError_t launch_ndr_vc3d_f32(const Problem& p, const BandGeom& g, const float* in, float* out,
                              const float* w, hipStream_t st) {
    return ndr::dispatch_vc3d<float>(p, g, in, out, w, st);
}
}  // namespace tvs
