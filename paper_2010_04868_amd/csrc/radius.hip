// Stencils of radius R > 1 (Section 1 classifies stencils by their number of
// points; Section 3.2's legality rule then asks for a skew s > R).
//
// plain_r: one Jacobi step per launch for any dimension, star or box, one
// thread per point, canonical offset order over {-R..R}^D.
//
// tstp1d_r: the 1D time-skewed pipeline for radius R.  A wave is a pipeline
// of up to 64 levels: lane l holds level t0+l+1 and at step q computes the
// point x = xb + q - s*l with s = R + 1.  The value of level l at x + R was
// computed by lane l-1 one step earlier, so each step every lane receives its
// predecessor's last output through a DPP shift (lane 0 receives the input
// value u[x + R]), and keeps the last 2R+1 values it received: exactly the
// window x-R .. x+R of the level below.  The input of a segment is staged in
// LDS; lane 0 takes it from a register holding 64 steps' worth, rotated down
// one lane per step.  Segments of L outputs overlap by k*R input points per
// side (a trapezoid in time), so pipelines never wait for each other.
#include <algorithm>
#include <cstring>

#include "kernels.hpp"

namespace tvs {
namespace {

__device__ __forceinline__ int64_t wrap64(int64_t i, int64_t n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Weights a plain step takes: at least kMaxPoints, else the stencil's count.
template <int D, bool BOX, int R>
constexpr int plain_cap() {
    return StencilR<D, BOX, R>::P > kMaxPoints ? StencilR<D, BOX, R>::P : kMaxPoints;
}

// VC: variable coefficients, the weight of offset q at point e is wts[q * N + e]
template <typename T, int D, bool BOX, int R, bool PER, bool VC = false>
__global__ __launch_bounds__(256) void plain_r(const T* __restrict__ in, T* __restrict__ out,
                                               int64_t n0, int64_t n1, int64_t n2,
                                               Coeffs<T, plain_cap<D, BOX, R>()> cf,
                                               const T* __restrict__ wts = nullptr) {
    using S = StencilR<D, BOX, R>;
    static_assert(S::P <= kMaxWeights, "weights");
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t ext[3] = {n0, n1, n2};
    int64_t total = 1;
    for (int a = 0; a < D; ++a) total *= ext[a];
    if (e >= total) return;
    int64_t c[3] = {0, 0, 0};
    int64_t rem = e;
    for (int a = D - 1; a >= 0; --a) {
        c[a] = rem % ext[a];
        rem /= ext[a];
    }
    bool fixed = false;
    for (int a = 0; a < D; ++a) fixed = fixed || c[a] < R || c[a] >= ext[a] - R;
    if (!PER && fixed) {
        out[e] = in[e];
        return;
    }
    T acc = 0;
    static_for<0, S::P>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        int64_t at = 0;
        for (int a = 0; a < D; ++a) {
            const int64_t v = PER ? wrap64(c[a] + S::off(q, a), ext[a]) : c[a] + S::off(q, a);
            at = at * ext[a] + v;
        }
        const T wq = VC ? wts[(int64_t)q * total + e] : cf.c[q];
        acc = term(acc, wq, in[at], q == 0);
    });
    out[e] = acc;
}

__device__ __forceinline__ float rot_down(float x) { return dpp<kDppWaveShl1>(x, x); }
__device__ __forceinline__ double rot_down(double x) { return dpp<kDppWaveShl1>(x, x); }

// One segment per wave, four waves per workgroup.  LDS per wave: the
// segment's input (u[xb-R .. xb+Q+R) at index 0 ..) plus a chunk of slack,
// then the top level's outputs.
// VC: variable coefficients, staged per wave in LDS after the outputs:
// wb[q * WL + (x - xb)] = wts[q * n + x] for the points the wave computes.
template <typename T, int R, bool PER, bool VC = false>
__global__ __launch_bounds__(256) void tstp1d_r(const T* __restrict__ in, T* __restrict__ out,
                                                int n, int k, int Lv, int nseg, int inlen,
                                                Coeffs<T> cf, const T* __restrict__ wts = nullptr,
                                                int WL = 0) {
    constexpr int s = R + 1;
    constexpr int WN = 2 * R + 1;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int sg = (int)blockIdx.x * 4 + w;
    T* inb = reinterpret_cast<T*>(smem_raw) + (size_t)w * (inlen + Lv + (VC ? WN * WL : 0));
    T* obuf = inb + inlen;
    T* wb = obuf + Lv;
    const bool live = sg < nseg;  // uniform per wave
    const int X0 = sg * Lv;
    const int xb = X0 - (k - 1) * R;               // level 1's first point
    const int Q = Lv + (k - 1) * (2 * R + 1);      // steps until the top level is done
    if (live)
        for (int i = lane; i < inlen; i += 64) {
            const int x = xb - R + i;  // inb[i] = u[x]
            T v = T(0);
            if (PER)
                v = in[(int)wrap64(((x % n) + n) % n, n)];
            else if (x >= 0 && x < n)
                v = in[x];
            inb[i] = v;
        }
    if (VC && live)
        for (int i = lane; i < WN * WL; i += 64) {
            const int q = i / WL, x = xb + i % WL;
            const int xi = PER ? ((x % n) + n) % n : min(max(x, 0), n - 1);
            wb[i] = wts[(int64_t)q * n + xi];
        }
    __syncthreads();
    if (live) {
        // window: wv[i] = level-below value at x - R + i; lane 0 starts with the inputs
        // xb-R .. xb+R-1 in wv[1..2R] (wv[0] is shifted out at the first step)
        T wv[WN];
#pragma unroll
        for (int i = 0; i < WN; ++i) wv[i] = lane == 0 && i >= 1 ? inb[i - 1] : T(0);
        T outv = T(0);
        for (int q0 = 0; q0 < Q; q0 += 64) {
            T tin = inb[2 * R + q0 + lane];  // u[xb + q + R] for q = q0 + lane
            static_for<0, 64>([&](auto mc) {
                constexpr int mm = decltype(mc)::value;
                const int q = q0 + mm;
                const T nv = shift_up<64>(outv, tin);  // the level below at x + R
                tin = rot_down(tin);
#pragma unroll
                for (int i = 0; i + 1 < WN; ++i) wv[i] = wv[i + 1];
                wv[WN - 1] = nv;
                const int x = xb + q - s * lane;
                T acc;
                if constexpr (VC) {
                    // lanes still filling the pipeline (x < xb) read any weight
                    const int o = max(x - xb, 0);
                    acc = wb[o] * wv[0];
#pragma unroll
                    for (int i = 1; i < WN; ++i) acc = acc + wb[i * WL + o] * wv[i];
                } else {
                    acc = cf.c[0] * wv[0];
#pragma unroll
                    for (int i = 1; i < WN; ++i) acc = acc + cf.c[i] * wv[i];
                }
                if (!PER) acc = (x < R || x >= n - R) ? wv[R] : acc;  // fixed ends
                outv = acc;
                if (lane == k - 1 && x >= X0 && x < X0 + Lv && x < n) obuf[x - X0] = outv;
            });
        }
    }
    __syncthreads();
    if (live)
        for (int i = lane; i < Lv && X0 + i < n; i += 64) out[X0 + i] = obuf[i];
}

// coeffs: the plan's coefficient buffer (kMaxWeights entries of T)
template <typename T, int D, bool BOX, int R>
hipError_t plain_r_go(const Problem& p, const T* in, T* out, const void* coeffs,
                      hipStream_t st) {
    const int64_t total = p.elems();
    const dim3 grid((unsigned)((total + 255) / 256));
    Coeffs<T, plain_cap<D, BOX, R>()> cf;
    std::memcpy(&cf, coeffs, sizeof cf);
    if (p.boundary == TVS_PERIODIC)
        hipLaunchKernelGGL((plain_r<T, D, BOX, R, true>), grid, dim3(256), 0, st, in, out,
                           p.dims[0], p.dims[1], p.dims[2], cf);
    else
        hipLaunchKernelGGL((plain_r<T, D, BOX, R, false>), grid, dim3(256), 0, st, in, out,
                           p.dims[0], p.dims[1], p.dims[2], cf);
    return hipGetLastError();
}

template <typename T>
hipError_t plain_radius_t(const Problem& p, const T* in, T* out, const void* cf,
                          hipStream_t st) {
    const bool box = p.shape == TVS_BOX;
    const int r = p.radius;
    if (p.ndim == 1) {
        if (r == 2) return plain_r_go<T, 1, false, 2>(p, in, out, cf, st);
        if (r == 3) return plain_r_go<T, 1, false, 3>(p, in, out, cf, st);
    } else if (p.ndim == 2) {
        if (r == 2) return box ? plain_r_go<T, 2, true, 2>(p, in, out, cf, st)
                               : plain_r_go<T, 2, false, 2>(p, in, out, cf, st);
        if (r == 3) return box ? plain_r_go<T, 2, true, 3>(p, in, out, cf, st)
                               : plain_r_go<T, 2, false, 3>(p, in, out, cf, st);
    } else {
        if (r == 2) return box ? plain_r_go<T, 3, true, 2>(p, in, out, cf, st)
                               : plain_r_go<T, 3, false, 2>(p, in, out, cf, st);
        if (r == 3 && !box) return plain_r_go<T, 3, false, 3>(p, in, out, cf, st);
    }
    return hipErrorInvalidValue;
}

int tstp1d_r_inlen(int R, int k, int Lv) {
    const int Q = Lv + (k - 1) * (2 * R + 1);
    const int chunks = (Q + 63) / 64;
    return 2 * R + 64 * chunks + 64;  // every read of a chunk's inputs stays inside
}

template <typename T, int R, bool PER>
hipError_t tstp1d_r_go(const Problem& p, const BandGeom& g, const T* in, T* out,
                       const Coeffs<T>& cf, hipStream_t st) {
    const int n = (int)p.dims[0];
    const int k = g.k, Lv = g.Lv;
    if (k < 1 || k > 64 || Lv < 1) return hipErrorInvalidValue;
    const int inlen = tstp1d_r_inlen(R, k, Lv);
    const size_t lds = (size_t)4 * (inlen + Lv) * sizeof(T);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void*)tstp1d_r<T, R, PER>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }
    const int nseg = (n + Lv - 1) / Lv;
    hipLaunchKernelGGL((tstp1d_r<T, R, PER>), dim3((unsigned)((nseg + 3) / 4)), dim3(256), lds, st,
                       in, out, n, k, Lv, nseg, inlen, cf);
    return hipGetLastError();
}

template <typename T>
hipError_t tstp1d_radius_t(const Problem& p, const BandGeom& g, const T* in, T* out,
                           const Coeffs<T>& cf, hipStream_t st) {
    const bool per = p.boundary == TVS_PERIODIC;
    if (p.radius == 2)
        return per ? tstp1d_r_go<T, 2, true>(p, g, in, out, cf, st)
                   : tstp1d_r_go<T, 2, false>(p, g, in, out, cf, st);
    if (p.radius == 3)
        return per ? tstp1d_r_go<T, 3, true>(p, g, in, out, cf, st)
                   : tstp1d_r_go<T, 3, false>(p, g, in, out, cf, st);
    return hipErrorInvalidValue;
}

// Variable coefficients: plain steps of radius 1..3 in any dimension.
template <typename T, int D, bool BOX, int R>
hipError_t plain_vc_go(const Problem& p, const T* in, T* out, const T* wts, hipStream_t st) {
    const int64_t total = p.elems();
    const dim3 grid((unsigned)((total + 255) / 256));
    const Coeffs<T, plain_cap<D, BOX, R>()> none{};
    if (p.boundary == TVS_PERIODIC)
        hipLaunchKernelGGL((plain_r<T, D, BOX, R, true, true>), grid, dim3(256), 0, st, in, out,
                           p.dims[0], p.dims[1], p.dims[2], none, wts);
    else
        hipLaunchKernelGGL((plain_r<T, D, BOX, R, false, true>), grid, dim3(256), 0, st, in, out,
                           p.dims[0], p.dims[1], p.dims[2], none, wts);
    return hipGetLastError();
}

template <typename T>
hipError_t plain_vc_t(const Problem& p, const T* in, T* out, const T* wts, hipStream_t st) {
    const bool box = p.shape == TVS_BOX;
    const int r = p.radius;
    if (p.ndim == 1) {
        if (r == 1) return plain_vc_go<T, 1, false, 1>(p, in, out, wts, st);
        if (r == 2) return plain_vc_go<T, 1, false, 2>(p, in, out, wts, st);
        if (r == 3) return plain_vc_go<T, 1, false, 3>(p, in, out, wts, st);
    } else if (p.ndim == 2) {
        if (r == 1) return box ? plain_vc_go<T, 2, true, 1>(p, in, out, wts, st)
                               : plain_vc_go<T, 2, false, 1>(p, in, out, wts, st);
        if (r == 2) return box ? plain_vc_go<T, 2, true, 2>(p, in, out, wts, st)
                               : plain_vc_go<T, 2, false, 2>(p, in, out, wts, st);
        if (r == 3) return box ? plain_vc_go<T, 2, true, 3>(p, in, out, wts, st)
                               : plain_vc_go<T, 2, false, 3>(p, in, out, wts, st);
    } else {
        if (r == 1) return box ? plain_vc_go<T, 3, true, 1>(p, in, out, wts, st)
                               : plain_vc_go<T, 3, false, 1>(p, in, out, wts, st);
        if (r == 2) return box ? plain_vc_go<T, 3, true, 2>(p, in, out, wts, st)
                               : plain_vc_go<T, 3, false, 2>(p, in, out, wts, st);
        if (r == 3 && !box) return plain_vc_go<T, 3, false, 3>(p, in, out, wts, st);
    }
    return hipErrorInvalidValue;
}

int vc_wl(int R, int k, int Lv) {
    const int Q = Lv + (k - 1) * (2 * R + 1);
    return 64 * ((Q + 63) / 64);  // every step of the last chunk reads inside
}

template <typename T, int R, bool PER>
hipError_t tstp1d_vc_go(const Problem& p, int k, int Lv, const T* in, T* out, const T* wts,
                        hipStream_t st) {
    const int n = (int)p.dims[0];
    if (k < 1 || k > 64 || Lv < 1) return hipErrorInvalidValue;
    const int inlen = tstp1d_r_inlen(R, k, Lv), WL = vc_wl(R, k, Lv);
    const size_t lds = (size_t)4 * (inlen + Lv + (2 * R + 1) * WL) * sizeof(T);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void*)tstp1d_r<T, R, PER, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }
    const int nseg = (n + Lv - 1) / Lv;
    const Coeffs<T> none{};
    hipLaunchKernelGGL((tstp1d_r<T, R, PER, true>), dim3((unsigned)((nseg + 3) / 4)), dim3(256),
                       lds, st, in, out, n, k, Lv, nseg, inlen, none, wts, WL);
    return hipGetLastError();
}

template <typename T>
hipError_t tstp1d_vc_t(const Problem& p, int k, int Lv, const T* in, T* out, const T* wts,
                       hipStream_t st) {
    const bool per = p.boundary == TVS_PERIODIC;
    switch (p.radius) {
        case 1: return per ? tstp1d_vc_go<T, 1, true>(p, k, Lv, in, out, wts, st)
                           : tstp1d_vc_go<T, 1, false>(p, k, Lv, in, out, wts, st);
        case 2: return per ? tstp1d_vc_go<T, 2, true>(p, k, Lv, in, out, wts, st)
                           : tstp1d_vc_go<T, 2, false>(p, k, Lv, in, out, wts, st);
        case 3: return per ? tstp1d_vc_go<T, 3, true>(p, k, Lv, in, out, wts, st)
                           : tstp1d_vc_go<T, 3, false>(p, k, Lv, in, out, wts, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t tstp1d_vc_lds_bytes(const Problem& p, int k, int Lv) {
    const int R = p.radius;
    return (size_t)4 * (tstp1d_r_inlen(R, k, Lv) + Lv + (2 * R + 1) * vc_wl(R, k, Lv)) *
           p.elem_bytes();
}

hipError_t launch_plain_varcoef(const Problem& p, const void* in, void* out, const void* wts,
                                hipStream_t st) {
    if (p.dtype == TVS_F64)
        return plain_vc_t<double>(p, (const double*)in, (double*)out, (const double*)wts, st);
    return plain_vc_t<float>(p, (const float*)in, (float*)out, (const float*)wts, st);
}

hipError_t launch_tstp1d_varcoef(const Problem& p, int k, int Lv, const void* in, void* out,
                                 const void* wts, hipStream_t st) {
    if (p.ndim != 1) return hipErrorInvalidValue;
    if (p.dtype == TVS_F64)
        return tstp1d_vc_t<double>(p, k, Lv, (const double*)in, (double*)out, (const double*)wts,
                                   st);
    return tstp1d_vc_t<float>(p, k, Lv, (const float*)in, (float*)out, (const float*)wts, st);
}

// Which (ndim, shape, radius > 1) combinations have kernels: every star and
// box of radius 2 and 3 with at most kMaxWeights points (all but the 3D
// radius-3 box, 343 points).
bool radius_supported(int ndim, int shape, int r) {
    if (r < 2 || r > 3) return false;
    return !(ndim == 3 && shape == TVS_BOX && r == 3);
}

// LDS bytes of a 1D radius-R band (four pipelines per workgroup).
size_t tstp1d_radius_lds_bytes(const Problem& p, int k, int Lv) {
    return (size_t)4 * (tstp1d_r_inlen(p.radius, k, Lv) + Lv) * p.elem_bytes();
}

hipError_t launch_plain_radius(const Problem& p, const void* in, void* out, const void* coeffs,
                               hipStream_t st) {
    if (p.dtype == TVS_F64)
        return plain_radius_t<double>(p, (const double*)in, (double*)out, coeffs, st);
    return plain_radius_t<float>(p, (const float*)in, (float*)out, coeffs, st);
}

hipError_t launch_tstp1d_radius(const Problem& p, const BandGeom& g, const void* in, void* out,
                                const void* coeffs, hipStream_t st) {
    if (p.ndim != 1) return hipErrorInvalidValue;
    if (p.dtype == TVS_F64)
        return tstp1d_radius_t<double>(p, g, (const double*)in, (double*)out,
                                       *(const Coeffs<double>*)coeffs, st);
    return tstp1d_radius_t<float>(p, g, (const float*)in, (float*)out,
                                  *(const Coeffs<float>*)coeffs, st);
}

}  // namespace tvs
