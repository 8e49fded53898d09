// 1D time-skewed pipeline: argument block and per-tile body, shared by the
// band kernel and the batch kernel.
#pragma once

#include "kernels.hpp"

namespace tvs {
namespace d1 {

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

// The pipelines of one "tile": 4 waves of 64/PL pipelines each.  Lanes of
// pipelines past the end return at once (whole pipelines only).
template <typename T, bool PER, int PL>
__device__ __forceinline__ void tstp1d_tile(const T* __restrict__ in, T* __restrict__ out,
                                            const Args1d& a, const Coeffs<T>& cf, int tile,
                                            int tid) {
    const int lane = tid & 63;
    const int j = lane % PL;  // lane j computes level j+1
    const int64_t seg = ((int64_t)tile * 4 + (tid >> 6)) * (64 / PL) + lane / PL;
    if (tid >= 256 || seg >= a.nseg) return;
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

}  // namespace d1
}  // namespace tvs
