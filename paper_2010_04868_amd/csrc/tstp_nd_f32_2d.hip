// Instantiation unit: time-skewed 2D Jacobi kernels, float storage.
#include "tstp_nd.hpp"

namespace tvs {
hipError_t launch_nd_f32_2d(const Problem& p, const BandGeom& g, const float* in, float* out,
                            const Coeffs<float>& cf, bool uniform, hipStream_t st) {
    return nd::launch_nd_impl<float, 2>(p, g, in, out, cf, uniform, st);
}
}  // namespace tvs
