// Time-skewed register pipeline for 2D Jacobi stencils.
//
// The same time skewing as the paper's temporal vectorization (Section 3.2:
// strip-mine time by k, skew the inner time loop against the outer space
// loop, Section 3.5), with the roles of lanes and registers exchanged: each
// lane carries all k time levels of its C columns as a software pipeline in
// registers, level j working one row behind level j-1 (s = 1: inside one
// lane the levels are evaluated in order, so level j may consume the row
// level j-1 produced in the same step), while the 64 lanes of a wave cover
// 64*C consecutive columns.  The level hand-off that Algorithm 3 performs
// with a rotate and a blend is a register rename here; the two neighbour
// columns a lane needs from the lanes beside it arrive by one DPP wave shift
// each way.  A wave is a complete tile: no LDS and no barriers.  Its edge
// lanes see garbage neighbours, which only reach points inside the k-wide
// halo that the trapezoid discards.  Each grid value crosses HBM once per
// band of k steps, with C consecutive elements per lane.
//
// Every point is computed with the canonical operation order (three running
// sums per point: stencil rows behind, at and ahead of it along the stream
// axis), and with equal weights a value's product with the weight is formed
// once and reused, which changes no bit.  The result is bit-identical to
// the naive sweep.
#pragma once

#include "kernels.hpp"

namespace tvs {
namespace reg {

struct ArgsReg {
    int nz, nx;       // stream axis, last axis
    int Wv;           // valid columns per tile (64*C - 2K)
    int Lv, Lin;      // valid rows per segment, rows read per segment
    int ntx;          // tiles along the last axis
    int ntiles;       // tiles in total
};

template <typename T, bool BOX, bool PER, int C, int K, bool UNI, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void tstp_reg2d(const T* __restrict__ in, T* __restrict__ out,
                                                  ArgsReg a, Coeffs<T> cf) {
    using St = Stencil<2, BOX>;
    constexpr int gm_b = St::group_begin(-1), gm_e = St::group_end(-1);
    constexpr int g0_b = St::group_begin(0), g0_e = St::group_end(0);
    constexpr int gp_b = St::group_begin(1), gp_e = St::group_end(1);
    constexpr int W = 64 * C;
    constexpr int DP = 2;  // input rows loaded ahead

    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;  // whole waves only
    const int bx = tile % a.ntx;
    const int bs = tile / a.ntx;
    const int x_org = bx * a.Wv - K;
    const int z_org = bs * a.Lv - K;
    const int xl0 = lane * C;
    const int nx = a.nx, nz = a.nz;

    // columns of this lane, wrapped or clamped once
    int gcol[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int gx = x_org + xl0 + c;
        gcol[c] = PER ? (int)wrap_idx(gx, nx) : (int)clamp_idx(gx, nx);
    }
    const bool border_tile =
        !PER && (x_org <= 0 || x_org + W - 1 >= nx - 1 || z_org <= 0 || z_org + a.Lin - 1 >= nz - 1);

    auto load_row = [&](int q, T* dst) __attribute__((always_inline)) {
        if (q >= a.Lin) return;
        int64_t gz = z_org + q;
        gz = PER ? wrap_idx(gz, nz) : clamp_idx(gz, nz);
        const T* row = in + gz * nx;
#pragma unroll
        for (int c = 0; c < C; ++c) dst[c] = row[gcol[c]];
    };

    T M[K][C], S[K][C];
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
        for (int c = 0; c < C; ++c) M[j][c] = S[j][c] = T(0);
    T pre[DP][C];
#pragma unroll
    for (int d = 0; d < DP; ++d) {
#pragma unroll
        for (int c = 0; c < C; ++c) pre[d][c] = T(0);
        load_row(d, pre[d]);
    }
    const T cu = cf.c[0];

    auto step = [&](int q, T* pr) __attribute__((always_inline)) {
        T vin[C];
#pragma unroll
        for (int c = 0; c < C; ++c) vin[c] = pr[c];
        load_row(q + DP, pr);
        static_for<0, K>([&](auto jc) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value;  // this level computes level j+1
            // v[i]: level-j value of column xl0-1+i in the row consumed now
            T v[C + 2];
            v[0] = dpp<kDppWaveShr1>(T(0), vin[C - 1]);
#pragma unroll
            for (int c = 0; c < C; ++c) v[1 + c] = vin[c];
            v[C + 1] = dpp<kDppWaveShl1>(T(0), vin[0]);
            if (UNI) {
#pragma unroll
                for (int i = 0; i < C + 2; ++i) v[i] = cu * v[i];
            }
            auto add = [&](T acc, auto qc, int c, bool first) __attribute__((always_inline)) -> T {
                constexpr int q2 = decltype(qc)::value;
                const T x = v[1 + c + St::off(q2, 1)];
                const T prod = UNI ? x : cf.c[q2] * x;
                return first ? prod : acc + prod;
            };
            const int row = q - j - 1;  // row emitted by level j+1
            const int64_t gz = (int64_t)z_org + row;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T f = M[j][c];
                static_for<gp_b, gp_e>([&](auto qc) __attribute__((always_inline)) { f = add(f, qc, c, false); });
                T m = S[j][c];
                static_for<g0_b, g0_e>([&](auto qc) __attribute__((always_inline)) { m = add(m, qc, c, false); });
                T s = T(0);
                static_for<gm_b, gm_e>([&](auto qc) __attribute__((always_inline)) {
                    s = add(s, qc, c, decltype(qc)::value == gm_b);
                });
                if (!PER && border_tile) {
                    // a fixed border point keeps its input value at every level
                    // (loaded for every point inside the tile-uniform branch, so
                    // that no divergent branch splits the unrolled pipeline)
                    const int gx = x_org + xl0 + c;
                    const bool fixed = (gz == 0 || gz == nz - 1 || gx == 0 || gx == nx - 1);
                    const T bv = in[clamp_idx(gz, nz) * nx + clamp_idx(gx, nx)];
                    f = fixed ? bv : f;
                }
                M[j][c] = m;
                S[j][c] = s;
                vin[c] = f;
            }
        });
        // vin now holds level K at row q-K
        const int row = q - K;
        const int64_t gz = (int64_t)z_org + row;
        if (row >= K && row < a.Lin - K && gz < nz) {
            T* o = out + gz * nx;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int xl = xl0 + c;
                const int gx = x_org + xl;
                if (xl >= K && xl < W - K && gx < nx) o[gx] = vin[c];
            }
        }
    };

    const int Q = a.Lin;
    for (int q = 0; q < Q; q += DP) {
        static_for<0, DP>([&](auto dc) __attribute__((always_inline)) {
            constexpr int d = decltype(dc)::value;
            if (q + d < Q) step(q + d, pre[d]);
        });
    }
}

template <typename T, int C, int K>
hipError_t launch_reg_impl(const Problem& p, const BandGeom& g, const T* in, T* out,
                           const Coeffs<T>& cf, bool uniform, hipStream_t st) {
    ArgsReg a{};
    a.nz = (int)p.dims[0];
    a.nx = (int)p.dims[1];
    a.Wv = 64 * C - 2 * K;
    a.Lv = g.Lv;
    a.Lin = g.Lv + 2 * K;
    a.ntx = (a.nx + a.Wv - 1) / a.Wv;
    const int nseg = (a.nz + a.Lv - 1) / a.Lv;
    a.ntiles = a.ntx * nseg;
    dim3 grid((unsigned)((a.ntiles + 3) / 4)), block(256);
    const bool box = p.shape == TVS_BOX, per = p.boundary == TVS_PERIODIC;
#define TVS_R(B, PR, U) \
    hipLaunchKernelGGL((tstp_reg2d<T, B, PR, C, K, U, 2>), grid, block, 0, st, in, out, a, cf)
    if (box) {
        if (per) { if (uniform) TVS_R(true, true, true); else TVS_R(true, true, false); }
        else { if (uniform) TVS_R(true, false, true); else TVS_R(true, false, false); }
    } else {
        if (per) { if (uniform) TVS_R(false, true, true); else TVS_R(false, true, false); }
        else { if (uniform) TVS_R(false, false, true); else TVS_R(false, false, false); }
    }
#undef TVS_R
    return hipGetLastError();
}

}  // namespace reg

// (K, C) pairs built for the register pipeline, per element type
bool reg2d_supported(int dtype, int k, int c);
hipError_t launch_reg2d(const Problem& p, const BandGeom& g, const void* in, void* out,
                        const void* coeffs, bool uniform, hipStream_t st);

}  // namespace tvs
