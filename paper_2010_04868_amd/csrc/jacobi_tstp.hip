// Band dispatch and geometry for the time-skewed Jacobi kernels.
#include <cstring>

#include "kernels.hpp"
#include "tstp_nd.hpp"

namespace tvs {

hipError_t launch_tstp1d(const Problem& p, const BandGeom& g, const void* in, void* out,
                         const void* coeffs, hipStream_t st);

bool tstp_supported(const Problem& p) {
    return p.dependence == TVS_JACOBI && p.radius == 1 && p.ndim >= 1 && p.ndim <= 3;
}

bool same_weight_bits(const double* c, int n) {
    for (int i = 1; i < n; ++i)
        if (std::memcmp(&c[i], &c[0], sizeof(double)) != 0) return false;
    return true;
}

bool band_geometry(const Problem& p, const Schedule& s, int k, BandGeom* g) {
    if (p.ndim >= 2 && p.radius > 1) return ndr_geometry(p, s, k, g);
    BandGeom r;
    r.k = k;
    r.lanemap = s.lanemap;
    if (k < 1) return false;
    if (p.ndim == 1) {
        r.pl = s.pl == 16 ? 16 : 64;
        if (k > r.pl) return false;
        r.Lv = s.l > 0 ? s.l : 256;
        r.nseg = (int)((p.dims[0] + r.Lv - 1) / r.Lv);
        r.NT = 256;
        *g = r;
        return true;
    }
    // the LDS pipeline addresses one stream-axis plane through a buffer
    // resource with 31-bit offsets
    const int64_t plane_bytes =
        (p.ndim == 3 ? p.dims[1] * p.dims[2] : p.dims[1]) * (int64_t)p.elem_bytes();
    if (plane_bytes >= (int64_t(1) << 31)) return false;
    r.C = s.c;
    if (r.C != 4 && r.C != 8 && r.C != 16) return false;
    r.W = s.w;
    if (r.W <= 2 * k || r.W % r.C) return false;
    r.Wv = r.W - 2 * k;
    if (p.ndim == 3) {
        r.H = s.h;
        if (r.H <= 2 * k) return false;
        r.Hv = r.H - 2 * k;
    } else {
        r.H = 1;
        r.Hv = 1;
    }
    r.G = r.H * r.W / r.C;
    r.NT = k * r.G;
    if (r.NT > 512) return false;
    // a thread stages at most 4 plane elements per step (k >= C/4)
    if ((int64_t)r.H * r.W > 4 * (int64_t)r.NT) return false;
    r.Lv = s.l > 0 ? s.l : 256;
    const int nstream = (int)p.dims[0];
    const int nxa = (int)p.dims[p.ndim - 1];
    r.ntx = (nxa + r.Wv - 1) / r.Wv;
    r.nty = p.ndim == 3 ? ((int)p.dims[1] + r.Hv - 1) / r.Hv : 1;
    r.nseg = (nstream + r.Lv - 1) / r.Lv;
    r.lds_bytes = tstp_nd_lds_bytes(p, r);
    if (r.lds_bytes > 160 * 1024) return false;
    *g = r;
    return true;
}

hipError_t launch_tstp_band(const Problem& p, const BandGeom& g, const void* in, void* out,
                            const void* coeffs, hipStream_t st) {
    if (p.ndim == 1) return launch_tstp1d(p, g, in, out, coeffs, st);
    if (p.radius > 1) return launch_tstp_ndr(p, g, in, out, coeffs, nullptr, st);
    if (p.rule == TVS_RULE_LIFE)
        return launch_nd_life_2d(p, g, (const uint32_t*)in, (uint32_t*)out, st);
    if (p.dtype == TVS_F64) {
        auto& cf = *(const Coeffs<double>*)coeffs;
        double cd[kMaxPoints];
        for (int q = 0; q < p.order; ++q) cd[q] = cf.c[q];
        const bool uni = same_weight_bits(cd, p.order);
        return p.ndim == 2 ? launch_nd_f64_2d(p, g, (const double*)in, (double*)out, cf, uni, st)
                           : launch_nd_f64_3d(p, g, (const double*)in, (double*)out, cf, uni, st);
    }
    auto& cf = *(const Coeffs<float>*)coeffs;
    double cd[kMaxPoints];
    for (int q = 0; q < p.order; ++q) cd[q] = cf.c[q];
    const bool uni = same_weight_bits(cd, p.order);
    return p.ndim == 2 ? launch_nd_f32_2d(p, g, (const float*)in, (float*)out, cf, uni, st)
                       : launch_nd_f32_3d(p, g, (const float*)in, (float*)out, cf, uni, st);
}

}  // namespace tvs
