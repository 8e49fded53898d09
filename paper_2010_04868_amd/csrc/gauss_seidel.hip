// In-place Gauss-Seidel sweeps (2D, star 5-point and box 9-point, radius 1).
//
// Section 3.4 ("Gauss-Seidel stencils"): one array holds the newest value of
// every point; a sweep visits points in lexicographic order, so neighbours
// that precede a point contribute this sweep's value and the centre and the
// neighbours after it the previous sweep's.  No single loop of the naive
// code can be vectorized, and diamond tiling is illegal; the paper uses
// parallelogram tiles and skews successive sweeps along the outer axis.
//
// GPU schedule:
//   * a work item is (band of 64 interior rows, sweep).  One wave runs it:
//     lane i owns row x0+i and walks the columns with a skew of sigma
//     columns per row (sigma = 1 for the star, 2 for the box), so every
//     value a lane needs from the row above was produced by lane i-1 in the
//     previous step and arrives by one DPP shift -- the wavefront relative of
//     temporal vectorization (Section 3.5);
//   * sweeps are skewed across waves: item (b, t) runs behind (b-1, t) and
//     behind (b, t-1) and (b+1, t-1), i.e. in the order of mu = 2t + b, the
//     parallelogram order; k sweeps are in flight in one launch, so each
//     band of rows is reused by k sweeps while it is still in cache;
//   * items are handed out by an atomic ticket in mu order to a persistent
//     grid of waves, so every dependence points to an earlier ticket held by
//     a running wave (no deadlock for any grid size); progress (columns
//     completed on the item's last row) is published with agent-scope
//     release/acquire, which also orders memory across the XCDs' L2 caches;
//   * every wait is bounded; on expiry the kernel records a status word and
//     the remaining waits return at once, so the launch always drains.
// Each point is updated exactly once per sweep, with the canonical operation
// order, after all of its "new" and before any of its "old" neighbours are
// overwritten, so the result is bit-identical to the naive lexicographic
// sweep.
#include "kernels.hpp"

namespace tvs {
namespace {

constexpr int kRows = 64;        // rows per band (one wave)
constexpr int kBlock = 8;        // steps whose loads are issued together
// Steps between dependency checks and progress updates.  Crossing the XCDs'
// separate L2 caches makes every agent-scope acquire and release expensive
// (an L2 invalidate or write-back), so they are done once per kSync steps;
// a dependent item then trails its producer by about kSync columns.
constexpr int kSync = 64;
static_assert(kSync % kBlock == 0, "sync interval");
constexpr long long kSpinLimit = 1ll << 22;  // ~seconds: far beyond any legitimate wait

struct GsArgs {
    int n0, n1;
    int nb;       // bands of interior rows
    int sweeps;   // sweeps in this launch
    int ncols;    // interior columns
    int nitems;
    int* ticket;
    int* status;
    int* progress;  // [sweeps][nb]
};

__device__ __forceinline__ int load_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *p >= need (or the launch has been aborted).  Uniform per wave.
// Relaxed polling: the caller issues one acquire fence after all its waits.
__device__ __forceinline__ void wait_at_least(const int* p, int need, int* status) {
    long long spins = 0;
    while (load_relaxed(p) < need) {
        if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
        if (++spins > kSpinLimit) {
            __hip_atomic_store(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

__global__ void gs_reset(int* ticket, int* progress, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *ticket = 0;
    for (; i < n; i += gridDim.x * blockDim.x) progress[i] = 0;
}

// item -> (band, sweep) in mu = 2*sweep + band order
__device__ void decode_item(int item, int nb, int sweeps, int* b, int* t) {
    int rem = item;
    for (int mu = 0;; ++mu) {
        int t_lo = mu - (nb - 1) > 0 ? (mu - (nb - 1) + 1) / 2 : 0;
        int t_hi = min(sweeps - 1, mu / 2);
        int cnt = t_hi >= t_lo ? t_hi - t_lo + 1 : 0;
        if (rem < cnt) {
            *t = t_lo + rem;
            *b = mu - 2 * *t;
            return;
        }
        rem -= cnt;
    }
}

// Value of lane 63 in every lane (wave-wide readlane).
template <typename T>
__device__ __forceinline__ T lane63(T v) {
    if constexpr (sizeof(T) == 8) {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
    }
}

// HR rows per lane: lane i owns rows x0+i, x0+64+i, ... of a band of 64*HR
// rows.  The halves form one wavefront (half h runs 64*SIG columns behind
// half h-1), so each lane carries HR independent dependency chains; the row
// above the first row of half h is the last row of half h-1, whose value
// comes from lane 63 by a readlane.
template <typename T, bool BOX, int HR>
__global__ __launch_bounds__(64) void gs2d(T* grid, GsArgs a, Coeffs<T> cf) {
    constexpr int SIG = BOX ? 2 : 1;
    constexpr int BR = kRows * HR;  // rows per band
    const int lane = threadIdx.x;
    const int64_t n1 = a.n1;
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(a.ticket, 1);
        item = __shfl(item, 0);
        if (item >= a.nitems) break;
        int b, t;
        decode_item(item, a.nb, a.sweeps, &b, &t);
        const int x0 = 1 + BR * b;
        const int rows = min(BR, a.n0 - 1 - x0);
        const int L = rows - 1;  // last active row of the band
        bool active[HR];
        T* row[HR];
        const T* row_s[HR];
        // registers per half: west (new), centre/east (old), north and south histories
        T Wv[HR], Cv[HR], Ev[HR], NWv[HR], Nv[HR], NEv[HR], SWv[HR], Sv[HR], SEv[HR], out[HR];
#pragma unroll
        for (int h = 0; h < HR; ++h) {
            const int ri = kRows * h + lane;
            active[h] = ri < rows;
            const int xr = x0 + (active[h] ? ri : 0);  // safe row for inactive lanes
            row[h] = grid + (int64_t)xr * n1;
            row_s[h] = grid + (int64_t)(xr + 1) * n1;
            Wv[h] = Cv[h] = out[h] = 0;
            Ev[h] = row[h][0];
            NWv[h] = Nv[h] = NEv[h] = grid[(int64_t)(xr - 1) * n1];
            SWv[h] = Sv[h] = SEv[h] = row_s[h][0];
        }
        const T* row_n = grid + (int64_t)(x0 - 1) * n1;  // lane 0's north row
        int* prog_self = a.progress + t * a.nb + b;
        const int* prog_north = b > 0 ? a.progress + t * a.nb + (b - 1) : nullptr;
        const int* prog_prev = t > 0 ? a.progress + (t - 1) * a.nb + b : nullptr;
        const int* prog_south =
            (t > 0 && b + 1 < a.nb) ? a.progress + (t - 1) * a.nb + (b + 1) : nullptr;

        // steps: row ri of the band is at column c = u - 1 - SIG*ri in [-1, ncols]
        const int U = a.ncols + 2 + SIG * L;
        for (int us = 0; us < U; us += kSync) {
          // columns the leading row (lane 0 of the first half) reaches in this interval
          const int cmax = us + kSync - 2;
          if (prog_prev) wait_at_least(prog_prev, min(a.ncols, cmax + 2), a.status);
          if (prog_south) wait_at_least(prog_south, min(a.ncols, cmax + 2), a.status);
          if (prog_north) wait_at_least(prog_north, min(a.ncols, cmax + SIG), a.status);
          // the producers' rows written before their progress stores are visible now
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          for (int u0 = us; u0 < us + kSync && u0 < U; u0 += kBlock) {
            T e_in[HR][kBlock], se_in[HR][kBlock], n_in[kBlock];
#pragma unroll
            for (int m = 0; m < kBlock; ++m) {
#pragma unroll
                for (int h = 0; h < HR; ++h) {
                    const int c = u0 + m - 1 - SIG * (kRows * h + lane);
                    const int ye = c + 2;
                    e_in[h][m] = se_in[h][m] = 0;
                    if (active[h] && c >= -1 && ye <= a.n1 - 1) {
                        e_in[h][m] = row[h][ye];
                        se_in[h][m] = row_s[h][ye];
                    }
                }
                const int c0 = u0 + m - 1 - SIG * lane;
                const int yn = c0 + SIG;
                n_in[m] = 0;
                if (lane == 0 && c0 >= -1 && yn <= a.n1 - 1) n_in[m] = row_n[yn];
            }
#pragma unroll
            for (int m = 0; m < kBlock; ++m) {
                // value of the row above, one column ahead of where the row
                // above was last step: lane i-1's last output; for lane 0 the
                // north row in memory (first half) or lane 63's last output of
                // the half before (taken before this step updates it)
                T nin[HR];
                nin[0] = shift_up<64>(out[0], n_in[m]);
#pragma unroll
                for (int h = 1; h < HR; ++h) nin[h] = shift_up<64>(out[h], lane63(out[h - 1]));
#pragma unroll
                for (int h = 0; h < HR; ++h) {
                    const int c = u0 + m - 1 - SIG * (kRows * h + lane);
                    if (c >= -1 && c <= a.ncols) {
                        if (BOX) {
                            NWv[h] = Nv[h];
                            Nv[h] = NEv[h];
                            NEv[h] = nin[h];
                            SWv[h] = Sv[h];
                            Sv[h] = SEv[h];
                            SEv[h] = se_in[h][m];
                        } else {
                            Nv[h] = nin[h];
                            Sv[h] = SEv[h];
                            SEv[h] = se_in[h][m];
                        }
                        Cv[h] = Ev[h];
                        Ev[h] = e_in[h][m];
                        T r = Cv[h];  // border columns pass their fixed value along
                        if (c >= 0 && c < a.ncols) {
                            if (BOX) {
                                r = cf.c[0] * NWv[h];
                                r = r + cf.c[1] * Nv[h];
                                r = r + cf.c[2] * NEv[h];
                                r = r + cf.c[3] * Wv[h];
                                r = r + cf.c[4] * Cv[h];
                                r = r + cf.c[5] * Ev[h];
                                r = r + cf.c[6] * SWv[h];
                                r = r + cf.c[7] * Sv[h];
                                r = r + cf.c[8] * SEv[h];
                            } else {
                                r = cf.c[0] * Nv[h];
                                r = r + cf.c[1] * Wv[h];
                                r = r + cf.c[2] * Cv[h];
                                r = r + cf.c[3] * Ev[h];
                                r = r + cf.c[4] * Sv[h];
                            }
                            if (active[h]) row[h][c + 1] = r;
                        }
                        Wv[h] = r;
                        out[h] = r;
                    }
                }
            }
          }
          // publish the columns completed on the band's last row
          const int done = min(a.ncols, max(0, us + kSync - 1 - SIG * L));
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          if (lane == 0) __hip_atomic_store(prog_self, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) __hip_atomic_store(prog_self, a.ncols, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename T>
hipError_t launch_gs_t(const Problem& p, T* grid, const Coeffs<T>& cf, int sweeps, int hr,
                       void* work, hipStream_t st) {
    if (hr != 1 && hr != 2) return hipErrorInvalidValue;
    GsArgs a{};
    a.n0 = (int)p.dims[0];
    a.n1 = (int)p.dims[1];
    a.ncols = a.n1 - 2;
    a.nb = (a.n0 - 2 + kRows * hr - 1) / (kRows * hr);
    a.sweeps = sweeps;
    a.nitems = a.nb * sweeps;
    int* w = (int*)work;
    a.ticket = w;
    a.status = w + 1;
    a.progress = w + 64;  // keep counters on their own cache lines
    const int nprog = a.nb * sweeps;
    hipLaunchKernelGGL(gs_reset, dim3((unsigned)std::min(1024, (nprog + 255) / 256 + 1)),
                       dim3(256), 0, st, a.ticket, a.progress, nprog);
    const int waves = std::min(a.nitems, 256 * 8);
    if (p.shape == TVS_BOX) {
        if (hr == 2) hipLaunchKernelGGL((gs2d<T, true, 2>), dim3(waves), dim3(64), 0, st, grid, a, cf);
        else hipLaunchKernelGGL((gs2d<T, true, 1>), dim3(waves), dim3(64), 0, st, grid, a, cf);
    } else {
        if (hr == 2) hipLaunchKernelGGL((gs2d<T, false, 2>), dim3(waves), dim3(64), 0, st, grid, a, cf);
        else hipLaunchKernelGGL((gs2d<T, false, 1>), dim3(waves), dim3(64), 0, st, grid, a, cf);
    }
    return hipGetLastError();
}

}  // namespace

size_t gs_work_bytes(const Problem& p, int sweeps) {
    const int nb = (int)((p.dims[0] - 2 + kRows - 1) / kRows);
    return (size_t)(64 + nb * sweeps + 64) * sizeof(int);
}

hipError_t launch_gs(const Problem& p, void* grid, const void* coeffs, int sweeps, int hr,
                     void* work, hipStream_t st) {
    if (p.dtype == TVS_F64)
        return launch_gs_t<double>(p, (double*)grid, *(const Coeffs<double>*)coeffs, sweeps, hr,
                                   work, st);
    return launch_gs_t<float>(p, (float*)grid, *(const Coeffs<float>*)coeffs, sweeps, hr, work,
                              st);
}

hipError_t gs_read_status(const void* work, int* status, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(status, (const int*)work + 1, sizeof(int),
                                  hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

}  // namespace tvs
