// Instantiations of the 2D register pipeline: (levels K, columns per lane C)
// pairs whose 2*K*C running sums fit the register file.
#include "tstp_reg2d.hpp"

namespace tvs {

bool reg2d_supported(int dtype, int k, int c) {
    if (dtype == TVS_F64)
        return (k == 8 && c == 4) || (k == 4 && c == 8) || (k == 16 && c == 2) || (k == 6 && c == 4);
    return (k == 8 && c == 8) || (k == 8 && c == 4) || (k == 16 && c == 4) || (k == 16 && c == 2);
}

hipError_t launch_reg2d(const Problem& p, const BandGeom& g, const void* in, void* out,
                        const void* coeffs, bool uniform, hipStream_t st) {
    if (p.dtype == TVS_F64) {
        auto& cf = *(const Coeffs<double>*)coeffs;
        auto i = (const double*)in;
        auto o = (double*)out;
        if (g.k == 8 && g.C == 4) return reg::launch_reg_impl<double, 4, 8>(p, g, i, o, cf, uniform, st);
        if (g.k == 4 && g.C == 8) return reg::launch_reg_impl<double, 8, 4>(p, g, i, o, cf, uniform, st);
        if (g.k == 16 && g.C == 2) return reg::launch_reg_impl<double, 2, 16>(p, g, i, o, cf, uniform, st);
        if (g.k == 6 && g.C == 4) return reg::launch_reg_impl<double, 4, 6>(p, g, i, o, cf, uniform, st);
        return hipErrorInvalidValue;
    }
    auto& cf = *(const Coeffs<float>*)coeffs;
    auto i = (const float*)in;
    auto o = (float*)out;
    if (g.k == 8 && g.C == 8) return reg::launch_reg_impl<float, 8, 8>(p, g, i, o, cf, uniform, st);
    if (g.k == 8 && g.C == 4) return reg::launch_reg_impl<float, 4, 8>(p, g, i, o, cf, uniform, st);
    if (g.k == 16 && g.C == 4) return reg::launch_reg_impl<float, 4, 16>(p, g, i, o, cf, uniform, st);
    if (g.k == 16 && g.C == 2) return reg::launch_reg_impl<float, 2, 16>(p, g, i, o, cf, uniform, st);
    return hipErrorInvalidValue;
}

}  // namespace tvs
