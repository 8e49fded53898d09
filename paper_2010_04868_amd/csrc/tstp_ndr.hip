// Geometry and dispatch of the 2D/3D band kernel for radius R > 1 and for
// variable coefficients (tstp_ndr.hpp).  The kernel instantiations live in
// tstp_ndr_{w,vc2d,vc3d}_{f64,f32}.hip.
#include "tstp_ndr.hpp"
#include "tstp_ndr_launch.hpp"

namespace tvs {

bool ndr_geometry(const Problem& p, const Schedule& s, int k, BandGeom* out, bool vc) {
    const int R = p.radius;
    if (p.ndim < 2 || R < 1 || R > 3 || k < 1) return false;
    // 3D: radius 1 and 2 (radius 3 runs plain steps: its 7 x (4 + 6) plane
    // values and 6 running sums per point exceed the registers of a lane);
    // boxes of radius 2 and above only in 2D
    if (p.ndim == 3 && (R == 3 || (R == 2 && p.shape == TVS_BOX))) return false;
    // the 2D radius-3 box (49 weights) runs plain steps
    if (p.order > kMaxPoints) return false;
    // 8 points per lane only for 2D constant weights
    if (s.c == 8 && (vc || p.ndim == 3)) return false;
    const int64_t plane_bytes =
        (p.ndim == 3 ? p.dims[1] * p.dims[2] : p.dims[1]) * (int64_t)p.elem_bytes();
    if (plane_bytes >= (int64_t(1) << 31)) return false;
    BandGeom g;
    g.k = k;
    g.lanemap = s.lanemap;
    g.C = s.c;
    if ((g.C != 4 && g.C != 8) || g.C < R) return false;
    g.W = s.w;
    if (g.W <= 2 * k * R || g.W % g.C) return false;
    g.Wv = g.W - 2 * k * R;
    if (p.ndim == 3) {
        g.H = s.h;
        if (g.H <= 2 * k * R) return false;
        g.Hv = g.H - 2 * k * R;
    } else {
        g.H = 1;
        g.Hv = 1;
    }
    g.G = g.H * g.W / g.C;
    g.NT = k * g.G;
    if (g.NT > 512) return false;
    if ((int64_t)g.H * g.W > 4 * (int64_t)g.NT) return false;  // at most 4 staged elements per thread
    g.Lv = s.l > 0 ? s.l : 256;
    g.ntx = ((int)p.dims[p.ndim - 1] + g.Wv - 1) / g.Wv;
    g.nty = p.ndim == 3 ? ((int)p.dims[1] + g.Hv - 1) / g.Hv : 1;
    g.nseg = ((int)p.dims[0] + g.Lv - 1) / g.Lv;
    g.lds_bytes = ndr::ndr_lds_bytes(p, g, vc);
    if (g.lds_bytes > 160 * 1024) return false;
    *out = g;
    return true;
}

hipError_t launch_tstp_ndr(const Problem& p, const BandGeom& g, const void* in, void* out,
                           const void* coeffs, const void* wts, hipStream_t st) {
    const bool vc = wts != nullptr;
    if (p.dtype == TVS_F64) {
        const auto& cf = *(const Coeffs<double>*)coeffs;
        auto i = (const double*)in;
        auto o = (double*)out;
        auto w = (const double*)wts;
        if (!vc) return launch_ndr_w_f64(p, g, i, o, cf, st);
        return p.ndim == 2 ? launch_ndr_vc2d_f64(p, g, i, o, w, st)
                           : launch_ndr_vc3d_f64(p, g, i, o, w, st);
    }
    const auto& cf = *(const Coeffs<float>*)coeffs;
    auto i = (const float*)in;
    auto o = (float*)out;
    auto w = (const float*)wts;
    if (!vc) return launch_ndr_w_f32(p, g, i, o, cf, st);
    return p.ndim == 2 ? launch_ndr_vc2d_f32(p, g, i, o, w, st)
                       : launch_ndr_vc3d_f32(p, g, i, o, w, st);
}

}  // namespace tvs
