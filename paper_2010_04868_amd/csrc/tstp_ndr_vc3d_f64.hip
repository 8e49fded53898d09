// Variable-coefficient 3D band kernels, double.
#include "tstp_ndr_launch.hpp"

namespace tvs {
hipError_t launch_ndr_vc3d_f64(const Problem& p, const BandGeom& g, const double* in, double* out,
                              const double* w, hipStream_t st) {
    return ndr::dispatch_vc3d<double>(p, g, in, out, w, st);
}
}  // namespace tvs
