// Instantiation unit: time-skewed Game of Life (B2S23) bands on 32-bit cells.
#include "tstp_nd.hpp"

namespace tvs {
hipError_t launch_nd_life_2d(const Problem& p, const BandGeom& g, const uint32_t* in,
                             uint32_t* out, hipStream_t st) {
    const Coeffs<uint32_t> none{};
    return nd::launch_nd_impl<uint32_t, 2, true>(p, g, in, out, none, false, st);
}
}  // namespace tvs
