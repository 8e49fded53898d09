// Plain Jacobi sweep: one time step per kernel launch.
//
// This is the naive (d+1)-loop algorithm of Section 1 (Algorithm 1 for the
// 1D 3-point case) with the space loops spread over the GPU: every step
// reads the whole grid once and writes it once (2 * element bytes per point
// update of HBM traffic).  It is the baseline the time-skewed kernels are
// measured against, so it is written to stream well: the stream axis is
// walked by each thread with a register window, the inner axes are
// coalesced and their neighbour re-reads hit in L1/L2.
#include <algorithm>

#include "kernels.hpp"

namespace tvs {
namespace {

template <typename T, bool PER>
__global__ __launch_bounds__(256) void plain1d(const T* __restrict__ in, T* __restrict__ out,
                                               int64_t n, Coeffs<T> cf) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!PER && (i == 0 || i == n - 1)) {
        out[i] = in[i];
        return;
    }
    int64_t im = i == 0 ? n - 1 : i - 1;
    int64_t ip = i == n - 1 ? 0 : i + 1;
    T acc = cf.c[0] * in[im];
    acc = acc + cf.c[1] * in[i];
    acc = acc + cf.c[2] * in[ip];
    out[i] = acc;
}

// 2D: thread = one column x, `RY` rows; every load of the strip is issued
// before the first update so that the memory system sees them all at once.
template <typename T, bool BOX, bool PER, int RY>
__global__ __launch_bounds__(256) void plain2d(const T* __restrict__ in, T* __restrict__ out,
                                               int n0, int n1, Coeffs<T> cf) {
    using S = Stencil<2, BOX>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n1) return;
    const int y0 = blockIdx.y * RY;
    const int xm = PER ? (x == 0 ? n1 - 1 : x - 1) : max(x - 1, 0);
    const int xp = PER ? (x == n1 - 1 ? 0 : x + 1) : min(x + 1, n1 - 1);
    const bool col_border = !PER && (x == 0 || x == n1 - 1);
    T w[RY + 2][3];
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        const int y = y0 - 1 + r;
        const int yy = PER ? (int)wrap_idx(y, n0) : (int)clamp_idx(y, n0);
        const T* row = in + (int64_t)yy * n1;
        w[r][0] = row[xm];
        w[r][1] = row[x];
        w[r][2] = row[xp];
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = y0 + r;
        if (y < n0) {
            T acc = 0;
            static_for<0, S::P>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                acc = term(acc, cf.c[q], w[r + 1 + S::off(q, 0)][1 + S::off(q, 1)], q == 0);
            });
            if (!PER && (col_border || y == 0 || y == n0 - 1)) acc = w[r + 1][1];
            out[(int64_t)y * n1 + x] = acc;
        }
    }
}

// Game of Life B2S23 (Section 3.4): the 2D 9-point box neighbourhood with
// the B2S23 rule in place of a weighted sum.  Same strip walk as plain2d.
// Sums are taken in unsigned 32-bit arithmetic (defined wrap-around; equal
// to the signed sum whenever that does not overflow).
template <bool PER, int RY>
__global__ __launch_bounds__(256) void plain_life(const uint32_t* __restrict__ in,
                                                  uint32_t* __restrict__ out, int n0, int n1) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n1) return;
    const int y0 = blockIdx.y * RY;
    const int xm = PER ? (x == 0 ? n1 - 1 : x - 1) : max(x - 1, 0);
    const int xp = PER ? (x == n1 - 1 ? 0 : x + 1) : min(x + 1, n1 - 1);
    const bool col_border = !PER && (x == 0 || x == n1 - 1);
    uint32_t w[RY + 2][3];
#pragma unroll
    for (int r = 0; r < RY + 2; ++r) {
        const int y = y0 - 1 + r;
        const int yy = PER ? (int)wrap_idx(y, n0) : (int)clamp_idx(y, n0);
        const uint32_t* row = in + (int64_t)yy * n1;
        w[r][0] = row[xm];
        w[r][1] = row[x];
        w[r][2] = row[xp];
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = y0 + r;
        if (y < n0) {
            const uint32_t c = w[r + 1][1];
            const uint32_t s = w[r][0] + w[r][1] + w[r][2] + w[r + 1][0] + w[r + 1][2] +
                               w[r + 2][0] + w[r + 2][1] + w[r + 2][2];
            uint32_t nv = (s == 2u || (c != 0u && s == 3u)) ? 1u : 0u;
            if (!PER && (col_border || y == 0 || y == n0 - 1)) nv = c;
            out[(int64_t)y * n1 + x] = nv;
        }
    }
}

// 3D: thread = one (y, x) column, `RZ` planes, all loads issued first.
template <typename T, bool BOX, bool PER, int RZ>
__global__ __launch_bounds__(256) void plain3d(const T* __restrict__ in, T* __restrict__ out,
                                               int n0, int n1, int n2, Coeffs<T> cf) {
    using S = Stencil<3, BOX>;
    const int x = blockIdx.x * 64 + threadIdx.x % 64;
    const int y = blockIdx.y * 4 + threadIdx.x / 64;
    if (x >= n2 || y >= n1) return;
    const int z0 = blockIdx.z * RZ;
    int xs[3], ys[3];
    for (int d = -1; d <= 1; ++d) {
        xs[d + 1] = PER ? (int)wrap_idx(x + d, n2) : (int)clamp_idx(x + d, n2);
        ys[d + 1] = PER ? (int)wrap_idx(y + d, n1) : (int)clamp_idx(y + d, n1);
    }
    const bool yx_border = !PER && (x == 0 || x == n2 - 1 || y == 0 || y == n1 - 1);
    T w[RZ + 2][3][3];
#pragma unroll
    for (int r = 0; r < RZ + 2; ++r) {
        const int z = z0 - 1 + r;
        const int zz = PER ? (int)wrap_idx(z, n0) : (int)clamp_idx(z, n0);
        const T* pl = in + (int64_t)zz * n1 * n2;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                // a star stencil reads only the centre column of the outer planes
                // and the cross of its own plane; the loads it does not need are
                // dead and removed by the compiler
                w[r][a][b] = pl[(int64_t)ys[a] * n2 + xs[b]];
            }
    }
#pragma unroll
    for (int r = 0; r < RZ; ++r) {
        const int z = z0 + r;
        if (z < n0) {
            T acc = 0;
            static_for<0, S::P>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                acc = term(acc, cf.c[q],
                           w[r + 1 + S::off(q, 0)][1 + S::off(q, 1)][1 + S::off(q, 2)], q == 0);
            });
            if (!PER && (yx_border || z == 0 || z == n0 - 1)) acc = w[r + 1][1][1];
            out[((int64_t)z * n1 + y) * n2 + x] = acc;
        }
    }
}

template <typename T>
hipError_t plain_step_t(const Problem& p, const T* in, T* out, const Coeffs<T>& cf,
                        hipStream_t st) {
    const bool per = p.boundary == TVS_PERIODIC;
    const bool box = p.shape == TVS_BOX;
    if (p.ndim == 1) {
        int64_t n = p.dims[0];
        dim3 grid((unsigned)((n + 255) / 256));
        if (per) hipLaunchKernelGGL((plain1d<T, true>), grid, dim3(256), 0, st, in, out, n, cf);
        else hipLaunchKernelGGL((plain1d<T, false>), grid, dim3(256), 0, st, in, out, n, cf);
    } else if (p.ndim == 2) {
        int n0 = (int)p.dims[0], n1 = (int)p.dims[1];
        constexpr int ry = 8;
        dim3 grid((unsigned)((n1 + 255) / 256), (unsigned)((n0 + ry - 1) / ry));
#define TVS_L2(B, PR) \
    hipLaunchKernelGGL((plain2d<T, B, PR, ry>), grid, dim3(256), 0, st, in, out, n0, n1, cf)
        if (box) { if (per) TVS_L2(true, true); else TVS_L2(true, false); }
        else { if (per) TVS_L2(false, true); else TVS_L2(false, false); }
#undef TVS_L2
    } else {
        int n0 = (int)p.dims[0], n1 = (int)p.dims[1], n2 = (int)p.dims[2];
        constexpr int rz = 4;
        dim3 grid((unsigned)((n2 + 63) / 64), (unsigned)((n1 + 3) / 4),
                  (unsigned)((n0 + rz - 1) / rz));
#define TVS_L3(B, PR) \
    hipLaunchKernelGGL((plain3d<T, B, PR, rz>), grid, dim3(256), 0, st, in, out, n0, n1, n2, cf)
        if (box) { if (per) TVS_L3(true, true); else TVS_L3(true, false); }
        else { if (per) TVS_L3(false, true); else TVS_L3(false, false); }
#undef TVS_L3
    }
    return hipGetLastError();
}

}  // namespace

// Device-to-device copy as a kernel (16-byte words, then the tail): unlike a
// runtime copy it records a plain kernel node when a run is captured in a
// graph.
__global__ void copy_words(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t nw,
                           const unsigned char* __restrict__ src_tail,
                           unsigned char* __restrict__ dst_tail, int tail) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < nw; i += (int64_t)gridDim.x * blockDim.x) dst[i] = src[i];
    if (i0 < tail) dst_tail[i0] = src_tail[i0];
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
    const int64_t nw = (int64_t)(bytes / 16);
    const int tail = (int)(bytes % 16);
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(8192, (nw + 255) / 256));
    hipLaunchKernelGGL(copy_words, dim3((unsigned)blocks), dim3(256), 0, st, (const uint4*)src,
                       (uint4*)dst, nw, (const unsigned char*)src + nw * 16,
                       (unsigned char*)dst + nw * 16, tail);
    return hipGetLastError();
}

hipError_t launch_plain_radius(const Problem& p, const void* in, void* out, const void* coeffs,
                               hipStream_t st);

hipError_t launch_plain_step(const Problem& p, const void* in, void* out, const void* coeffs,
                             hipStream_t st) {
    if (p.radius > 1) return launch_plain_radius(p, in, out, coeffs, st);
    if (p.rule == TVS_RULE_LIFE) {
        const int n0 = (int)p.dims[0], n1 = (int)p.dims[1];
        constexpr int ry = 8;
        dim3 grid((unsigned)((n1 + 255) / 256), (unsigned)((n0 + ry - 1) / ry));
        if (p.boundary == TVS_PERIODIC)
            hipLaunchKernelGGL((plain_life<true, ry>), grid, dim3(256), 0, st,
                               (const uint32_t*)in, (uint32_t*)out, n0, n1);
        else
            hipLaunchKernelGGL((plain_life<false, ry>), grid, dim3(256), 0, st,
                               (const uint32_t*)in, (uint32_t*)out, n0, n1);
        return hipGetLastError();
    }
    if (p.dtype == TVS_F64)
        return plain_step_t<double>(p, (const double*)in, (double*)out,
                                    *(const Coeffs<double>*)coeffs, st);
    return plain_step_t<float>(p, (const float*)in, (float*)out, *(const Coeffs<float>*)coeffs,
                               st);
}

}  // namespace tvs
