// Instantiation units of the radius-R / variable-coefficient band kernel:
// one per precision and kind, compiled in parallel.  Each dispatches on the
// stencil (dimension, shape, radius) at run time.
#pragma once

#include "tstp_ndr.hpp"

namespace tvs {

// weighted stencils of radius 2 and 3 (2D and 3D stars, the 2D radius-2 box)
hipError_t launch_ndr_w_f64(const Problem&, const BandGeom&, const double*, double*,
                            const Coeffs<double>&, hipStream_t);
hipError_t launch_ndr_w_f32(const Problem&, const BandGeom&, const float*, float*,
                            const Coeffs<float>&, hipStream_t);
// variable coefficients of radius 1..3 in 2D and 3D
hipError_t launch_ndr_vc2d_f64(const Problem&, const BandGeom&, const double*, double*,
                               const double*, hipStream_t);
hipError_t launch_ndr_vc2d_f32(const Problem&, const BandGeom&, const float*, float*,
                               const float*, hipStream_t);
hipError_t launch_ndr_vc3d_f64(const Problem&, const BandGeom&, const double*, double*,
                               const double*, hipStream_t);
hipError_t launch_ndr_vc3d_f32(const Problem&, const BandGeom&, const float*, float*,
                               const float*, hipStream_t);

namespace ndr {

// The weighted radius-R band kernels: every radius_supported stencil of
// radius 2 and 3 in 2D, the radius-2 star in 3D (ndr_geometry)
template <typename T>
hipError_t dispatch_w(const Problem& p, const BandGeom& g, const T* in, T* out,
                      const Coeffs<T>& cf, hipStream_t st) {
    const bool box = p.shape == TVS_BOX;
    const int r = p.radius;
    if (p.ndim == 2) {
        if (r == 2) return box ? launch_ndr_impl<T, 2, true, 2, false>(p, g, in, out, cf, nullptr, st)
                               : launch_ndr_impl<T, 2, false, 2, false>(p, g, in, out, cf, nullptr, st);
        if (r == 3 && !box) return launch_ndr_impl<T, 2, false, 3, false>(p, g, in, out, cf, nullptr, st);
    } else if (p.ndim == 3 && !box && r == 2) {
        return launch_ndr_impl<T, 3, false, 2, false>(p, g, in, out, cf, nullptr, st);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_vc2d(const Problem& p, const BandGeom& g, const T* in, T* out, const T* w,
                         hipStream_t st) {
    const Coeffs<T> none{};
    const bool box = p.shape == TVS_BOX;
    switch (p.radius) {
        case 1: return box ? launch_ndr_impl<T, 2, true, 1, true>(p, g, in, out, none, w, st)
                           : launch_ndr_impl<T, 2, false, 1, true>(p, g, in, out, none, w, st);
        case 2: return box ? launch_ndr_impl<T, 2, true, 2, true>(p, g, in, out, none, w, st)
                           : launch_ndr_impl<T, 2, false, 2, true>(p, g, in, out, none, w, st);
        case 3: return box ? hipErrorInvalidValue
                           : launch_ndr_impl<T, 2, false, 3, true>(p, g, in, out, none, w, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t dispatch_vc3d(const Problem& p, const BandGeom& g, const T* in, T* out, const T* w,
                         hipStream_t st) {
    const Coeffs<T> none{};
    const bool box = p.shape == TVS_BOX;
    switch (p.radius) {
        case 1: return box ? launch_ndr_impl<T, 3, true, 1, true>(p, g, in, out, none, w, st)
                           : launch_ndr_impl<T, 3, false, 1, true>(p, g, in, out, none, w, st);
        case 2: return box ? hipErrorInvalidValue
                           : launch_ndr_impl<T, 3, false, 2, true>(p, g, in, out, none, w, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ndr
}  // namespace tvs
