// Time-skewed temporal pipeline for 1D Jacobi stencils.
//
// The paper's central idea (Section 3.2, "Algorithm"): a vector holds points
// of successive time levels, t_{i+1} - t_i = 1, placed s apart along the
// swept space axis, so that one pass over the grid advances it by as many
// steps as the vector has lanes.  Here the vector is a pipeline of PL lanes
// (a 16-lane DPP row or a whole 64-lane wave) sweeping one segment.  Lane j
// holds level j+1.  Each step a lane receives the level-j value one
// position further along from lane j-1 by a single DPP shift -- the
// rotate-and-blend of Algorithm 3 as one cross-lane move, with the fresh
// level-0 value entering lane 0 through the DPP "old" operand -- finishes
// one level-(j+1) point and hands it on.  Level-0 values arrive as a
// coalesced "bottom vector" once per PL steps, broadcast lane by lane; the
// last active lane writes the band's top level.  Each level works s = 2
// positions behind the one before it (legality: s > max dx/dt, Section 3.2).
// Segments overlap by k points per side (a trapezoid in time), so pipelines
// never wait for each other.  Every point is computed with the canonical
// operation order, so the result is bit-identical to the naive sweep.
#include "tstp1d.hpp"

namespace tvs {
using namespace d1;
namespace {

// ---------------------------------------------------------------------------
// 1D
// ---------------------------------------------------------------------------
template <typename T, bool PER, int PL>
__global__ __launch_bounds__(256) void tstp1d(const T* __restrict__ in, T* __restrict__ out,
                                              Args1d a, Coeffs<T> cf) {
    tstp1d_tile<T, PER, PL>(in, out, a, cf, blockIdx.x, threadIdx.x);
}

template <typename T, bool PER>
hipError_t launch_1d(const Problem& p, const BandGeom& g, const T* in, T* out,
                     const Coeffs<T>& cf, hipStream_t st) {
    Args1d a{};
    a.n = p.dims[0];
    a.k = g.k;
    a.Lv = g.Lv;
    a.nseg = (a.n + g.Lv - 1) / g.Lv;
    const int pipes_per_block = 4 * (64 / g.pl);
    dim3 grid((unsigned)((a.nseg + pipes_per_block - 1) / pipes_per_block)), block(256);
    if (g.pl == 16)
        hipLaunchKernelGGL((tstp1d<T, PER, 16>), grid, block, 0, st, in, out, a, cf);
    else
        hipLaunchKernelGGL((tstp1d<T, PER, 64>), grid, block, 0, st, in, out, a, cf);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_tstp1d(const Problem& p, const BandGeom& g, const void* in, void* out,
                         const void* coeffs, hipStream_t st) {
    const bool per = p.boundary == TVS_PERIODIC;
    if (p.dtype == TVS_F64) {
        auto& cf = *(const Coeffs<double>*)coeffs;
        return per ? launch_1d<double, true>(p, g, (const double*)in, (double*)out, cf, st)
                   : launch_1d<double, false>(p, g, (const double*)in, (double*)out, cf, st);
    }
    auto& cf = *(const Coeffs<float>*)coeffs;
    return per ? launch_1d<float, true>(p, g, (const float*)in, (float*)out, cf, st)
               : launch_1d<float, false>(p, g, (const float*)in, (float*)out, cf, st);
}

}  // namespace tvs
