// Weighted radius-2/3 band kernels, double.
#include "tstp_ndr_launch.hpp"

namespace tvs {
hipError_t launch_ndr_w_f64(const Problem& p, const BandGeom& g, const double* in, double* out,
                           const Coeffs<double>& cf, hipStream_t st) {
    return ndr::dispatch_w<double>(p, g, in, out, cf, st);
}
}  // namespace tvs
