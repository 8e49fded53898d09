// Instantiation unit: time-skewed 2D Jacobi kernels, double storage.
#include "tstp_nd.hpp"

namespace tvs {
hipError_t launch_nd_f64_2d(const Problem& p, const BandGeom& g, const double* in, double* out,
                            const Coeffs<double>& cf, bool uniform, hipStream_t st) {
    return nd::launch_nd_impl<double, 2>(p, g, in, out, cf, uniform, st);
}
}  // namespace tvs
