// Order in which the 2D Gauss-Seidel kernel's waves take their items
// (band b, sweep t): by mu = 2t + b, the wavefront of Section 3.4's
// parallelogram tiling, in which every item an item waits for comes
// earlier.  Host and device, so that the order is checked on the CPU.
#pragma once

namespace tvs {
namespace gs {

__host__ __device__ inline int imin(int a, int b) { return a < b ? a : b; }

// Sweeps of band b = mu - 2t present at wavefront mu: t in [t_lo, t_hi].
__host__ __device__ inline void mu_range(int mu, int nb, int sweeps, int* t_lo, int* t_hi) {
    *t_lo = mu - (nb - 1) > 0 ? (mu - (nb - 1) + 1) / 2 : 0;
    *t_hi = imin(sweeps - 1, mu / 2);
}

// item -> (band, sweep): the item-th of all nb x sweeps items in mu order
// (within one mu, by increasing sweep).
__host__ __device__ inline void decode_item(int item, int nb, int sweeps, int* b, int* t) {
    int rem = item;
    for (int mu = 0;; ++mu) {
        int t_lo, t_hi;
        mu_range(mu, nb, sweeps, &t_lo, &t_hi);
        const int cnt = t_hi >= t_lo ? t_hi - t_lo + 1 : 0;
        if (rem < cnt) {
            *t = t_lo + rem;
            *b = mu - 2 * *t;
            return;
        }
        rem -= cnt;
    }
}

}  // namespace gs
}  // namespace tvs
