// Instantiation unit: time-skewed 3D Jacobi kernels, double storage.
#include "tstp_nd.hpp"

namespace tvs {
hipError_t launch_nd_f64_3d(const Problem& p, const BandGeom& g, const double* in, double* out,
                            const Coeffs<double>& cf, bool uniform, hipStream_t st) {
    return nd::launch_nd_impl<double, 3>(p, g, in, out, cf, uniform, st);
}
}  // namespace tvs
