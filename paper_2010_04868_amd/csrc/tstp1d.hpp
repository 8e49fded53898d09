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

// One pipeline step body, specialised for whether the pipelines of this wave
// touch a fixed end of the grid (interior waves carry no test for it).
//
// Level 0: a bottom vector holds the level-0 values of PL steps (one per
// lane).  It is written to LDS one block ahead, and lane 0 of each pipeline
// reads the value of step m+D there D steps early, straight into the
// register that the DPP shift's "old" operand takes, so the step's
// dependency chain is only the shift, one product and one sum.
// Output: the top level (lane k-1 of a pipeline) finishes one point per
// step.  Every lane writes its value to LDS at a compile-time offset each
// step -- lane k-1 into its pipeline's output row, the others into a scrap
// area -- so no step needs a branch; after PL steps the wave reads the
// output rows back (lane i: pipeline i / PL, step i % PL) and stores them
// with one coalesced store.  Blocks always run all PL steps: steps past the
// last one compute values that are never stored.
template <typename T, bool PER, int PL, bool BORDER>
__device__ __forceinline__ void tstp1d_run(const T* __restrict__ in, T* __restrict__ out,
                                           const Args1d& a, const Coeffs<T>& cf, int64_t s0,
                                           int j, int lane, T* obuf, T* scrap, T* bottom) {
    constexpr int D = 4;  // steps between an LDS read of a level-0 value and its use
    static_assert(D < PL, "read-ahead within two blocks");
    const int k = a.k;
    const int64_t n = a.n;
    const int Lin = a.Lv + 2 * k;
    const int Q = Lin + k - 1;  // steps until the last level has drained
    const T c0 = cf.c[0], c1 = cf.c[1], c2 = cf.c[2];

    auto load_block = [&](int blk) -> T {
        const int local = blk * PL + j;
        if (local >= Lin) return T(0);
        int64_t g = s0 + local;
        g = PER ? wrap_idx(g, n) : clamp_idx(g, n);
        return in[g];
    };
    // lane k-1 writes its pipeline's output row; the rest write scrap
    T* wbase = j == k - 1 ? obuf + (lane - j) : scrap + lane;
    // level-0 values: bottom[par][lane], read by pipeline row (lane - j) + m
    const int prow = lane - j;

    T accA = 0, accB = 0, prev = 0, fin = 0;
    T cur = load_block(0);
    T nxt = load_block(1);
    bottom[lane] = cur;
    T inj[D];
#pragma unroll
    for (int d = 0; d < D; ++d) inj[d] = bottom[prow + d];
    const int nblk = (Q + PL - 1) / PL;
    for (int blk = 0; blk < nblk; ++blk) {
        T after = load_block(blk + 2);  // prefetch two bottom vectors ahead
        const int par = blk & 1;
        T* bcur = bottom + par * 64 + prow;
        T* bnxt = bottom + (par ^ 1) * 64 + prow;
        bottom[(par ^ 1) * 64 + lane] = nxt;  // next block's level 0
        static_for<0, PL>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            // rotate + blend: lane j <- lane j-1's last output, lane 0 <- level 0
            const T v = shift_up<PL>(fin, inj[m % D]);
            T f = accB + c2 * v;   // level j+1 at pos-1: last term
            accB = accA + c1 * v;  // level j+1 at pos: middle term
            accA = c0 * v;         // level j+1 at pos+1: first term
            if constexpr (BORDER) {
                const int q = blk * PL + m;
                const int pos = q - 2 * j;  // local position of v (level j)
                const int64_t g = s0 + pos - 1;
                if (g == 0 || g == n - 1) f = prev;  // fixed end
            }
            prev = v;
            fin = f;
            wbase[m] = f;
            // level-0 value of step m + D
            if constexpr (m + D < PL) inj[m % D] = bcur[m + D];
            else inj[m % D] = bnxt[m + D - PL];
        });
        // store the top level's outputs of these PL steps
        const int q = blk * PL + lane % PL;
        const int loc = q - 2 * (k - 1) - 1;
        const int64_t g = s0 + loc;
        const T r = obuf[lane];
        if (q < Q && loc >= k && loc < Lin - k && g < n) out[g] = r;
        cur = nxt;
        nxt = after;
    }
}

// The pipelines of one "tile": 4 waves of 64/PL pipelines each.  Lanes of
// pipelines past the end return at once (whole pipelines only).
template <typename T, bool PER, int PL>
__device__ __forceinline__ void tstp1d_tile(const T* __restrict__ in, T* __restrict__ out,
                                            const Args1d& a, const Coeffs<T>& cf, int tile,
                                            int tid) {
    // per wave: an output row per pipeline (64 slots), 128 scrap slots and
    // two bottom vectors (128 slots)
    __shared__ T lds[4][64 + 128 + 128];
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int j = lane % PL;  // lane j computes level j+1
    const int64_t seg0 = ((int64_t)tile * 4 + wave) * (64 / PL);  // first pipeline of the wave
    const int64_t seg = seg0 + lane / PL;
    if (tid >= 256 || seg >= a.nseg) return;
    const int64_t s0 = seg * a.Lv - a.k;  // global position of local position 0
    T* obuf = lds[wave];
    T* scrap = lds[wave] + 64;
    T* bottom = lds[wave] + 192;
    if constexpr (PER) {
        tstp1d_run<T, PER, PL, false>(in, out, a, cf, s0, j, lane, obuf, scrap, bottom);
    } else {
        // the wave's pipelines read positions [seg0*Lv - k, (seg0 + 64/PL)*Lv + k)
        const int64_t lo = seg0 * a.Lv - a.k;
        const int64_t hi = (seg0 + 64 / PL) * (int64_t)a.Lv + a.k;
        const bool border = lo <= 0 || hi >= a.n - 1;
        if (border)
            tstp1d_run<T, PER, PL, true>(in, out, a, cf, s0, j, lane, obuf, scrap, bottom);
        else
            tstp1d_run<T, PER, PL, false>(in, out, a, cf, s0, j, lane, obuf, scrap, bottom);
    }
}

}  // namespace d1
}  // namespace tvs
