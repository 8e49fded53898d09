// Instantiation unit: time-skewed 3D Jacobi kernels, float storage.
#include "tstp_nd.hpp"

namespace tvs {
hipError_t launch_nd_f32_3d(const Problem& p, const BandGeom& g, const float* in, float* out,
                            const Coeffs<float>& cf, bool uniform, hipStream_t st) {
    return nd::launch_nd_impl<float, 3>(p, g, in, out, cf, uniform, st);
}
}  // namespace tvs
