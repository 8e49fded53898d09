// Shared host/device definitions for the tvstencil HIP library.
//
// Every translation unit of the library is compiled with
// -ffp-contract=off: a point update is a chain of separately rounded
// products and sums in canonical offset order, and no compiler pass may fuse
// or reorder it.  That, and nothing else, is what makes every schedule below
// produce the same bits as the naive loops.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <utility>

#include "../../include/tvstencil.h"

namespace tvs {

// ---------------------------------------------------------------------------
// Problem description (host side).
// ---------------------------------------------------------------------------
constexpr int kMaxDim = 3;
constexpr int kMaxPoints = 27;    // weights a band kernel takes (the radius-1 box in 3D)
constexpr int kMaxWeights = 125;  // weights of any stencil (the radius-2 box in 3D)

struct Problem {
    int ndim = 0;
    int64_t dims[kMaxDim] = {1, 1, 1};
    int dtype = TVS_F64, shape = TVS_STAR, order = 0, dependence = TVS_JACOBI,
        boundary = TVS_DIRICHLET;
    int radius = 1;
    int rule = TVS_RULE_WEIGHTED;  // TVS_RULE_LIFE: B2S23 on int32 cells (2D box, Jacobi)
    int64_t elems() const {
        int64_t n = 1;
        for (int a = 0; a < ndim; ++a) n *= dims[a];
        return n;
    }
    size_t elem_bytes() const { return dtype == TVS_F64 ? 8 : 4; }
    size_t bytes() const { return (size_t)elems() * elem_bytes(); }
    int64_t updated_points() const {
        int64_t n = 1;
        for (int a = 0; a < ndim; ++a)
            n *= boundary == TVS_PERIODIC ? dims[a] : dims[a] - 2 * radius;
        return n;
    }
};

struct Schedule {
    int method = TVS_METHOD_PLAIN;
    int k = 1;        // levels per band
    int s = 2;        // skew between successive levels (stream positions)
    int w = 0;        // tile extent along the last axis, halo included
    int h = 1;        // 3D: tile extent along axis 1, halo included
    int l = 0;        // stream segment length (valid outputs)
    int c = 1;        // points per lane along the last axis
    int lanemap = 0;  // 0: levels fastest within a wave; 1: columns fastest
    int pl = 64;      // 1D: lanes per pipeline (16 = one DPP row, 64 = a wave)
    int kern = 0;     // kernel kind: 0 = levels in lane groups with LDS planes (the only one)
};

// Error reporting: thread-local message + code.
int set_error(int code, const std::string& msg);
void clear_error();

#define TVS_HIP_TRY(expr)                                                              \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess)                                                          \
            return ::tvs::set_error(TVS_E_DEVICE, std::string(#expr) + ": " +          \
                                                      hipGetErrorString(_e));          \
    } while (0)

// ---------------------------------------------------------------------------
// Coefficients as a kernel argument (canonical order, storage precision).
// ---------------------------------------------------------------------------
// N: capacity (the plain steps of stencils of more than kMaxPoints points
// take exactly their own count).
template <typename T, int N = kMaxPoints>
struct Coeffs {
    T c[N];
};

// ---------------------------------------------------------------------------
// Canonical offsets at compile time.
//
// Offsets are the vectors of {-1,0,1}^D (star: at most one non-zero
// component) listed lexicographically with axis 0 most significant.  The
// point update is c[0]*v[0] followed by "+ c[q]*v[q]" in that order.
// ---------------------------------------------------------------------------
template <int D, bool BOX>
struct Stencil {
    static constexpr int P = BOX ? (D == 1 ? 3 : D == 2 ? 9 : 27) : 2 * D + 1;

    // component `a` of offset number q
    static constexpr int off(int q, int a) {
        int total = 1;
        for (int i = 0; i < D; ++i) total *= 3;
        int seen = 0;
        for (int lin = 0; lin < total; ++lin) {
            int d[3] = {0, 0, 0};
            int rem = lin, nz = 0;
            for (int i = D - 1; i >= 0; --i) {
                d[i] = rem % 3 - 1;
                rem /= 3;
                nz += d[i] != 0;
            }
            if (!BOX && nz > 1) continue;
            if (seen == q) return d[a];
            ++seen;
        }
        return 0;
    }
    // first and one-past-last canonical index whose axis-0 offset is d0
    static constexpr int group_begin(int d0) {
        for (int q = 0; q < P; ++q)
            if (off(q, 0) == d0) return q;
        return P;
    }
    static constexpr int group_end(int d0) {
        int e = group_begin(d0);
        while (e < P && off(e, 0) == d0) ++e;
        return e;
    }
};

// Canonical offsets of radius R: the vectors of {-R..R}^D (star: at most one
// non-zero component) in lexicographic order, axis 0 most significant.
template <int D, bool BOX, int R>
struct StencilR {
    static constexpr int side = 2 * R + 1;
    static constexpr int P = BOX ? (D == 1 ? side : D == 2 ? side * side : side * side * side)
                                 : 2 * D * R + 1;
    static constexpr int off(int q, int a) {
        int total = 1;
        for (int i = 0; i < D; ++i) total *= side;
        int seen = 0;
        for (int lin = 0; lin < total; ++lin) {
            int d[3] = {0, 0, 0};
            int rem = lin, nz = 0;
            for (int i = D - 1; i >= 0; --i) {
                d[i] = rem % side - R;
                rem /= side;
                nz += d[i] != 0;
            }
            if (!BOX && nz > 1) continue;
            if (seen == q) return d[a];
            ++seen;
        }
        return 0;
    }
    // first and one-past-last canonical index whose axis-0 offset is d0: the
    // offsets of one axis-0 offset are a contiguous run of the order
    static constexpr int group_begin(int d0) {
        for (int q = 0; q < P; ++q)
            if (off(q, 0) == d0) return q;
        return P;
    }
    static constexpr int group_end(int d0) {
        int e = group_begin(d0);
        while (e < P && off(e, 0) == d0) ++e;
        return e;
    }
};

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(static_cast<F&&>(f));
    }
}

// One canonical term: acc = first ? c*v : acc + c*v.  The product is rounded
// on its own before the sum (contraction is disabled for the library).
template <typename T>
__device__ __forceinline__ T term(T acc, T c, T v, bool first) {
    T prod = c * v;
    return first ? prod : acc + prod;
}

// ---------------------------------------------------------------------------
// Cross-lane moves (DPP).  A 64-bit value moves as two 32-bit halves.
// ---------------------------------------------------------------------------
// DPP control encodings (GFX9 family, which includes gfx950).
constexpr int kDppRowShr1 = 0x111;   // lane i <- lane i-1 within each row of 16
constexpr int kDppRowShl1 = 0x101;   // lane i <- lane i+1 within each row of 16
constexpr int kDppWaveShr1 = 0x138;  // lane i <- lane i-1 across the wave
constexpr int kDppWaveShl1 = 0x130;  // lane i <- lane i+1 across the wave
constexpr int kDppRowBcast15 = 0x142;  // row r+1 <- lane 15 of row r

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int dpp32(int old, int src) {
    return __builtin_amdgcn_update_dpp(old, src, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp(float old, float src) {
    return __int_as_float(dpp32<CTRL, ROW_MASK>(__float_as_int(old), __float_as_int(src)));
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp(double old, double src) {
    long long o = __double_as_longlong(old), s = __double_as_longlong(src);
    int lo = dpp32<CTRL, ROW_MASK>((int)(o & 0xffffffffll), (int)(s & 0xffffffffll));
    int hi = dpp32<CTRL, ROW_MASK>((int)(o >> 32), (int)(s >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Shift one lane up along a pipeline: lane i receives x from lane i-1; the
// first lane of each pipeline receives `first`.  PL = 16: a DPP row is a
// pipeline (four per wave); PL = 64: the whole wave is one pipeline.
template <int PL, typename T>
__device__ __forceinline__ T shift_up(T x, T first) {
    if constexpr (PL == 16) {
        return dpp<kDppRowShr1>(first, x);
    } else {
        return dpp<kDppWaveShr1>(first, x);
    }
}

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global load and store, which would stall the pipeline on
// the prefetch it has just issued; the pipeline exchanges data through LDS
// alone, so an LDS-scoped release/acquire around s_barrier is sufficient.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Periodic / clamped index.
// Raw buffer access (gfx9 resource layout, stride 0).  An access whose byte
// offset is not below the resource's size is dropped by the hardware (a
// store) or returns zero (a load), without touching memory.  Kernels mask
// lanes and rows that way instead of branching, so every wave of a pipeline
// issues the same memory instructions in every step and the compiler can
// count the outstanding ones exactly (a branch that may skip a load or a
// store forces it to wait for all of them).
// Offset of a masked lane: far beyond any resource the kernels build (their
// sizes stay below 2^31 bytes) and safe from wrap-around in the range check.
constexpr uint32_t kBufOOB = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    static_assert(sizeof(T) == 8 || sizeof(T) == 4, "element size");
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, T v) {
    static_assert(sizeof(T) == 8 || sizeof(T) == 4, "element size");
    if constexpr (sizeof(T) == 8) {
        using V2 = unsigned int __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, (int)off, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)off, 0,
                                              0);
    }
}

// Workgroups of a launch are dispatched to the 8 XCDs round robin (block b
// runs on XCD b mod 8).  This maps block b to a tile index such that every
// XCD processes one contiguous range of tiles, so tiles that share a halo
// mostly run on the same XCD and meet in its L2.  It is a bijection on
// [0, n) for every n.
__host__ __device__ __forceinline__ int xcd_block(int b, int n) {
    constexpr int X = 8;
    const int x = b % X, i = b / X;
    const int per = n / X, rem = n % X;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

__host__ __device__ __forceinline__ int64_t wrap_idx(int64_t i, int64_t n) {
    i %= n;
    return i < 0 ? i + n : i;
}
__host__ __device__ __forceinline__ int64_t clamp_idx(int64_t i, int64_t n) {
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

}  // namespace tvs
