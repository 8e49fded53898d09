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
#include "kernels.hpp"

namespace tvs {
namespace {

// ---------------------------------------------------------------------------
// 1D
// ---------------------------------------------------------------------------
struct Args1d {
    int64_t n;
    int k;     // levels in this band (<= PL)
    int Lv;    // valid outputs per pipeline
    int64_t nseg;
};

template <int PL, typename T>
__device__ __forceinline__ T lane_value(T v, int m) {
    if constexpr (PL == 64) {
        if constexpr (sizeof(T) == 8) {
            long long b = __double_as_longlong(v);
            int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), m);
            int hi = __builtin_amdgcn_readlane((int)(b >> 32), m);
            return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
        } else {
            return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), m));
        }
    } else {
        return __shfl(v, m, PL);
    }
}

template <typename T, bool PER, int PL>
__global__ __launch_bounds__(256) void tstp1d(const T* __restrict__ in, T* __restrict__ out,
                                              Args1d a, Coeffs<T> cf) {
    const int lane = threadIdx.x & 63;
    const int j = lane % PL;  // lane j computes level j+1
    const int64_t seg = ((int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * (64 / PL) +
                        lane / PL;
    if (seg >= a.nseg) return;  // whole pipelines only (PL divides 64)
    const int k = a.k;
    const int64_t n = a.n;
    const int64_t s0 = seg * a.Lv - k;  // global position of local position 0
    const int Lin = a.Lv + 2 * k;
    const int Q = Lin + k - 1;          // steps until the last level has drained
    const T c0 = cf.c[0], c1 = cf.c[1], c2 = cf.c[2];

    auto load_block = [&](int blk) -> T {
        const int local = blk * PL + j;
        if (local >= Lin) return T(0);
        int64_t g = s0 + local;
        g = PER ? wrap_idx(g, n) : clamp_idx(g, n);
        return in[g];
    };

    T accA = 0, accB = 0, prev = 0, fin = 0;
    T cur = load_block(0);
    T nxt = load_block(1);
    for (int blk = 0; blk * PL < Q; ++blk) {
        T after = load_block(blk + 2);  // prefetch two bottom vectors ahead
        static_for<0, PL>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const int q = blk * PL + m;
            if (q < Q) {
                // level-0 value for lane 0 of the pipeline at local position q
                const T inject = lane_value<PL>(cur, m);
                // rotate + blend: lane j <- lane j-1's last output, lane 0 <- inject
                const T v = shift_up<PL>(fin, inject);
                const int pos = q - 2 * j;  // local position of v (level j)
                T f = accB + c2 * v;        // level j+1 at pos-1: last term
                accB = accA + c1 * v;       // level j+1 at pos: middle term
                accA = c0 * v;              // level j+1 at pos+1: first term
                if (!PER) {
                    const int64_t g = s0 + pos - 1;
                    if (g == 0 || g == n - 1) f = prev;  // fixed end
                }
                prev = v;
                fin = f;
                if (j == k - 1) {
                    const int loc = pos - 1;
                    const int64_t g = s0 + loc;
                    if (loc >= k && loc < Lin - k && g < n) out[g] = f;
                }
            }
        });
        cur = nxt;
        nxt = after;
    }
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
