// Time-skewed temporal pipeline for 2D and 3D Jacobi stencils of radius R
// (1..3) and for variable coefficients.
//
// The same scheme as the radius-1 band kernel (tstp_nd.hpp): axis 0 is the
// stream axis (Section 3.2 vectorizes the outermost space loop in time), a
// workgroup owns a tile and a stream segment for a band of k levels, lane
// group j holds level t0+j, levels hand rows over through LDS planes, and a
// lane carries running sums that are contiguous runs of the canonical order.
// What changes with the radius:
//
//   * a level reads one row of the level below per step and contributes to
//     the 2R+1 points whose stencils contain that row: the point R rows ahead
//     receives its first run of terms (axis-0 offset -R), the point R rows
//     behind its last (offset +R) and is finished.  So a point carries 2R
//     running sums across steps, kept in a ring indexed by its row modulo 2R;
//   * the skew is s = 2R positions per level.  Legality (Section 3.2, s > max
//     dx/dt) needs s >= R + 1; s = 2R also makes a row's ring slot the same
//     for every level (row = step + R - 2R j), so the ring index is a
//     compile-time constant of the unrolled step loop.  A level then reads the
//     row its predecessor emitted R steps earlier, so each level keeps its
//     last R + 1 emitted rows (R + 1 LDS slots, the slot a uniform counter);
//   * a lane reads C + 2R values per plane row, and 2R + 1 plane rows in 3D;
//     tiles and stream segments overlap by k R points per side;
//   * a fixed (Dirichlet) point keeps its value: the lane emits point row p-R
//     at the step it reads row p, and its value at the level below is the
//     centre value the lane read R steps earlier (a ring of R raw rows).
//
// Variable coefficients (VC): the weight of offset q at point e is
// wts[q * N + e] (N grid points).  Every level needs the same weights, each
// at a different step.  A 2D radius-1 band with one staged element per
// thread stages them in an LDS ring: at step q the workgroup stores the P
// weights of point row q+1 of its tile (loaded two steps earlier with
// coalesced row loads), and a level reads the weights of the point rows it
// updates from the ring, which holds the 2Rk + 2 rows in flight (level j at
// step q updates rows q - 2Rj .. q + 2R - 2Rj).  So each weight crosses HBM
// once per band instead of once per level.  Elsewhere (3D: a plane of
// weights per row) the lane that forms a term loads its weight.  Products are never shared between terms: every term is its own weight
// times its value, in canonical order, so the result is bit-identical to
// the naive sweep.
#pragma once

#include <algorithm>
#include <type_traits>

#include "kernels.hpp"
#include "tstp_nd.hpp"

namespace tvs {
namespace ndr {

using nd::ArgsNd;

template <int R>
struct Unroll {
    static constexpr int DP = R == 3 ? 3 : 4;            // prefetch depth (steps)
    static constexpr int U = R == 3 ? 6 : 4;             // lcm(2R, DP): steps per loop body
    static_assert(U % (2 * R) == 0 && U % DP == 0, "compile-time ring indices");
};

// Whether a band stages its variable coefficients in an LDS ring: 2D radius
// 1 with one staged element per thread (a thread then loads at most P <= 9
// weights of a row; at radius 2 the weights in flight spill registers).
constexpr bool ndr_weight_ring(bool vc, int D, int R, int npt) {
    return vc && D == 2 && R == 1 && npt == 1;
}

template <typename T, int D, bool BOX, int R, bool PER, int C, int NPT, bool VC>
__global__ __launch_bounds__(512) void tstp_ndr(const T* __restrict__ in, T* __restrict__ out,
                                                ArgsNd a, Coeffs<T> cf,
                                                const T* __restrict__ wts) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    using St = StencilR<D, BOX, R>;
    constexpr int P = St::P;
    static_assert(P <= kMaxPoints, "weights");
    static_assert(C >= R, "a lane's halo comes from its two neighbour groups");
    constexpr int NR = D == 3 ? 2 * R + 1 : 1;  // plane rows a lane reads
    constexpr int NX = C + 2 * R;               // values per plane row
    constexpr int MID = D == 3 ? R : 0;         // the lane's own plane row
    constexpr int NA = 2 * R;                   // running sums carried per point
    constexpr int SL = R + 1;                   // LDS slots per level
    constexpr int DP = Unroll<R>::DP;
    constexpr int U = Unroll<R>::U;
    // weights staged in an LDS ring; a thread loads at most P weights per step
    constexpr bool WR = ndr_weight_ring(VC, D, R, NPT);
    constexpr int DPW = 2;                     // weight rows are loaded DPW steps ahead
    static_assert(U % DPW == 0, "compile-time weight prefetch slot");
    constexpr int NWL = WR ? P : 1;

    const int tid = threadIdx.x;
    const int k = a.k;
    const int S = a.S;
    const int Wp = a.Wp;
    int b = nd::tile_order(blockIdx.x, a);
    const int bx = b % a.ntx;
    b /= a.ntx;
    const int by = b % a.nty;
    const int bs = b / a.nty;
    const int x_org = bx * a.Wv - k * R;
    const int y_org = D == 3 ? by * a.Hv - k * R : 0;
    const int z_org = bs * a.Lv - k * R;

    int j, g;
    if (a.lanemap == 0) {
        j = 1 + tid % k;
        g = tid / k;
    } else {
        j = 1 + tid / a.G;
        g = tid % a.G;
    }
    const int ly = D == 3 ? g / a.Gx : 0;  // lane's tile row (3D)
    const int gx = g - ly * a.Gx;          // lane group within the row
    const int lx = gx * C;                 // lane's first tile column

    bool border_tile = false;
    if (!PER) {
        border_tile = x_org < R || x_org + a.W - 1 >= a.nx - R || z_org < R ||
                      z_org + a.Lin - 1 >= a.nz - R;
        if (D == 3) border_tile = border_tile || y_org < R || y_org + a.H - 1 >= a.ny - R;
    }
    const int gy_lane = y_org + ly;
    const bool y_border = D == 3 && !PER && (gy_lane < R || gy_lane >= a.ny - R);

    // LDS plane of level l (0..k) in slot r (0..R)
    auto plane = [&](int l, int r) -> T* { return lds + (r * (k + 1) + l) * a.PSP; };
    // WR: weight ring after the planes, NSW slots of P rows (transposed
    // layout, row stride Wp); slot of point row r is r mod NSW
    const int NSW = 2 * R * k + 2;
    T* const wring = lds + (k + 1) * SL * a.PSP;
    const int n_lds = (k + 1) * SL * a.PSP + (WR ? NSW * P * Wp : 0);
    for (int e = tid; e < n_lds; e += a.NT) lds[e] = T(0);

    // staging of level 0 (loads) and level k (stores), as in the radius-1 kernel
    const int PS = a.H * a.W;
    int st_lds[NPT];
    uint32_t ld_off[NPT], st_off[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int e = tid + i * a.NT;
        st_lds[i] = -1;
        ld_off[i] = st_off[i] = kBufOOB;
        if (e < PS) {
            const int yl = D == 3 ? e / a.W : 0;
            const int xl = e - yl * a.W;
            const int ox = x_org + xl, oy = y_org + yl;
            const int gxx = PER ? (int)wrap_idx(ox, a.nx) : (int)clamp_idx(ox, a.nx);
            const int gyy = D == 3 ? (PER ? (int)wrap_idx(oy, a.ny) : (int)clamp_idx(oy, a.ny)) : 0;
            st_lds[i] = (D == 3 ? (yl + R) * Wp : 0) + (xl % C) * S + xl / C + 1;
            ld_off[i] = (uint32_t)(gyy * a.nx + gxx) * (uint32_t)sizeof(T);
            const int kr = k * R;
            const bool valid = xl >= kr && xl < a.W - kr && ox < a.nx &&
                               (D != 3 || (yl >= kr && yl < a.H - kr && oy < a.ny));
            if (valid) st_off[i] = (uint32_t)(oy * a.nx + ox) * (uint32_t)sizeof(T);
        }
    }
    const uint32_t plane_bytes = (uint32_t)a.ny * (uint32_t)a.nx * (uint32_t)sizeof(T);
    auto row_ptr = [&](const T* base, int row) {
        return (const T*)((const char*)base + (uint64_t)(uint32_t)row * plane_bytes);
    };
    int ld_row = PER ? (int)wrap_idx(z_org, a.nz) : 0;
    auto issue_load = [&](int q, T* dst) {
        int gz;
        if (PER) {
            gz = ld_row;
            ld_row = ld_row + 1 == a.nz ? 0 : ld_row + 1;
        } else {
            gz = min(max(z_org + q, 0), a.nz - 1);
        }
        const auto rs = buf_rsrc(row_ptr(in, gz), q < a.Lin ? plane_bytes : 0u);
#pragma unroll
        for (int i = 0; i < NPT; ++i) dst[i] = buf_load<T>(rs, ld_off[i]);
    };

    // VC: the lane's weight addresses.  Column and row (3D) of each of its
    // points, wrapped (periodic) or clamped (points outside the grid feed
    // only points that are never stored).
    int wx[VC ? C : 1];
    int wy = 0;
    if constexpr (VC) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int ox = x_org + lx + c;
            wx[c] = PER ? (int)wrap_idx(ox, a.nx) : (int)clamp_idx(ox, a.nx);
        }
        if (D == 3) wy = PER ? (int)wrap_idx(gy_lane, a.ny) : (int)clamp_idx(gy_lane, a.ny);
    }
    const int64_t npts = (int64_t)a.nz * a.ny * a.nx;
    // WR: this thread's share of a weight row (P terms x W columns): element
    // e = tid + i*NT is term e / W at tile column e % W
    const int nwl = WR ? (P * a.W + a.NT - 1) / a.NT : 0;
    int wl_lds[NWL];
    int64_t wl_off[NWL];
    T prew[DPW][NWL];
    if constexpr (WR) {
#pragma unroll
        for (int i = 0; i < NWL; ++i) {
            const int e = tid + i * a.NT;
            wl_lds[i] = -1;
            wl_off[i] = 0;
            if (i < nwl && e < P * a.W) {
                const int q2 = e / a.W, xl = e - q2 * a.W;
                const int ox = x_org + xl;
                const int gxx = PER ? (int)wrap_idx(ox, a.nx) : (int)clamp_idx(ox, a.nx);
                wl_lds[i] = q2 * Wp + (xl % C) * S + xl / C + 1;
                wl_off[i] = (int64_t)q2 * npts + gxx;
            }
#pragma unroll
            for (int d = 0; d < DPW; ++d) prew[d][i] = T(0);
        }
    }
    // WR: load the weights of point row r (tile-local) into dst
    auto issue_wload = [&](int r, T* dst) {
        int zr = z_org + r;
        zr = PER ? (int)wrap_idx(zr, a.nz) : (int)clamp_idx(zr, a.nz);
        const int64_t row = (int64_t)zr * a.nx;
#pragma unroll
        for (int i = 0; i < NWL; ++i)
            if (wl_lds[i] >= 0) dst[i] = wts[wl_off[i] + row];
    };
    auto wslot_of = [&](int r) { return ((r % NSW) + NSW) % NSW; };

    T Acc[NA][C];
    T prevc[R][C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int r = 0; r < NA; ++r) Acc[r][c] = T(0);
#pragma unroll
        for (int r = 0; r < R; ++r) prevc[r][c] = T(0);
    }
    T pre[DP][NPT];
#pragma unroll
    for (int d = 0; d < DP; ++d)
#pragma unroll
        for (int i = 0; i < NPT; ++i) pre[d][i] = T(0);

    const int row_off = D == 3 ? ly * Wp : 0;  // padded row ly + R holds tile row ly
    int wslot = 0;                              // LDS slot written at this step (q mod (R+1))

    auto step = [&](int q, T* pr, auto bt, auto dc) {
        constexpr bool BT = !PER && decltype(bt)::value;
        constexpr int d = decltype(dc)::value;  // q mod U
        const int rslot = wslot + 1 == SL ? 0 : wslot + 1;   // (q - R) mod (R + 1)
        const int oslot = wslot == 0 ? SL - 1 : wslot - 1;   // (q - 1) mod (R + 1)
        // level 0: row q enters LDS; row q + DP is requested
        if (q < a.Lin) {
            T* pl = plane(0, wslot);
#pragma unroll
            for (int i = 0; i < NPT; ++i)
                if (st_lds[i] >= 0) pl[st_lds[i]] = pr[i];
        }
        issue_load(q + DP, pr);
        // level k emitted row q - 1 - 2Rk at step q - 1: store it
        {
            const int row = q - 1 - 2 * R * k;
            const int gz = z_org + row;
            const bool ok = row >= k * R && row < a.Lin - k * R && gz < a.nz;
            const T* pl = plane(k, oslot);
            const auto rs = buf_rsrc(row_ptr(out, ok ? gz : 0), ok ? plane_bytes : 0u);
#pragma unroll
            for (int i = 0; i < NPT; ++i)
                buf_store<T>(rs, st_off[i], pl[st_lds[i] < 0 ? 0 : st_lds[i]]);
        }
        // level j reads row p of level j-1 (emitted R steps ago) and emits
        // row p - R
        const int p = q + R - 2 * R * j;
        if constexpr (WR) {
            // point row q + 1 enters the weight ring (loaded DPW steps ago);
            // row q + 1 + DPW is requested
            T* wr = wring + wslot_of(q + 1) * P * Wp;
#pragma unroll
            for (int i = 0; i < NWL; ++i)
                if (wl_lds[i] >= 0) wr[wl_lds[i]] = prew[d % DPW][i];
            issue_wload(q + 1 + DPW, prew[d % DPW]);
        } else if constexpr (VC) {
            // the weight addresses are formed afresh each step: hoisted out
            // of the loop, the P x C loop-invariant parts would each hold a
            // 64-bit register pair for the whole band
#pragma unroll
            for (int c = 0; c < C; ++c) asm volatile("" : "+v"(wx[c]));
        }
        if (!BT || (p >= 0 && p < a.Lin)) {
            const T* src = plane(j - 1, rslot) + row_off;
            // weight of term q2 for the point c whose axis-0 offset to row p
            // is that term's (its row is p - off(q2, 0))
            auto weight = [&](auto qc, int c) -> T {
                constexpr int q2 = decltype(qc)::value;
                if constexpr (WR) {
                    const T* wr = wring + wslot_of(p - St::off(q2, 0)) * P * Wp;
                    return wr[q2 * Wp + c * S + gx + 1];
                } else if constexpr (VC) {
                    int zr = z_org + p - St::off(q2, 0);
                    zr = PER ? (int)wrap_idx(zr, a.nz) : (int)clamp_idx(zr, a.nz);
                    const int64_t at = (int64_t)q2 * npts +
                                       ((int64_t)zr * a.ny + wy) * a.nx + wx[c];
                    return wts[at];
                } else {
                    return cf.c[q2];
                }
            };
            const int gz_out = z_org + p - R;
            const bool z_border = !PER && (gz_out < R || gz_out >= a.nz - R);
            const bool emit = !BT || p >= R;
            T* dst = plane(j, wslot) + (D == 3 ? row_off + R * Wp : 0) + gx + 1;
            // ring slot of the point whose axis-0 offset to row p is dd
            auto slot = [](int dd) { return ((d + R - dd) % NA + NA) % NA; };
            // f: the point R rows behind, finished by the terms of offset +R;
            // s: the point R rows ahead, started by the terms of offset -R
            // (both use the same ring slot)
            T f[C], s[C], cen[C];  // cen: the raw centre values of row p (fixed points)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                f[c] = Acc[slot(R)][c];
                s[c] = T(0);
            }
            // One plane row at a time (3D: axis-1 offsets -R..R in order; 2D:
            // the one row).  Within a run of one axis-0 offset the terms are
            // ordered by axis-1 offset, so taking the rows in order keeps
            // every point's canonical order.
            static_for<0, NR>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                constexpr int a1 = D == 3 ? r - R : 0;

                const T* rs = src + r * Wp;
                T v[NX];
#pragma unroll
                for (int i = 0; i < NX; ++i) {
                    const bool need = BOX || r == MID || (i >= R && i < R + C);
                    if (!need) continue;
                    const int e = i - R;                     // column offset from lx
                    const int grp = e < 0 ? -1 : (e >= C ? 1 : 0);
                    const int sl = e - grp * C;              // element within the group
                    v[i] = rs[sl * S + gx + grp + 1];
                }
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    // VC: keep each point's weight loads next to their use
                    // (hoisted over the whole step they would hold P x C
                    // registers)
                    if constexpr (VC && !WR) __builtin_amdgcn_sched_barrier(0);
                    static_for<-R, R + 1>([&](auto dc2) {
                        constexpr int dd = decltype(dc2)::value;
                        T acc = dd == R ? f[c] : dd == -R ? s[c] : Acc[slot(dd)][c];
                        static_for<St::group_begin(dd), St::group_end(dd)>([&](auto qc) {
                            constexpr int q2 = decltype(qc)::value;
                            if constexpr (D == 2 || St::off(q2, 1) == a1) {
                                constexpr int col = D == 3 ? St::off(q2, 2) : St::off(q2, 1);
                                const T prod = weight(qc, c) * v[R + c + col];
                                acc = (dd == -R && q2 == St::group_begin(-R)) ? prod : acc + prod;
                            }
                        });
                        if (dd == R) f[c] = acc;
                        else if (dd == -R) s[c] = acc;
                        else Acc[slot(dd)][c] = acc;
                    });
                    if constexpr (BT && r == MID) cen[c] = v[R + c];
                }
            });
#pragma unroll
            for (int c = 0; c < C; ++c) {
                Acc[slot(-R)][c] = s[c];
                if constexpr (BT) {
                    // a fixed point keeps its value: the centre value this
                    // lane read R steps ago
                    const int gxc = x_org + lx + c;
                    const bool fixed = z_border || y_border || gxc < R || gxc >= a.nx - R;
                    if (emit) dst[c * S] = fixed ? prevc[d % R][c] : f[c];
                    prevc[d % R][c] = cen[c];
                } else {
                    if (emit) dst[c * S] = f[c];
                }
            }
        }
        lds_barrier();
        wslot = wslot + 1 == SL ? 0 : wslot + 1;
    };

    lds_barrier();  // LDS zeroed
#pragma unroll
    for (int d = 0; d < DP; ++d) issue_load(d, pre[d]);
    if constexpr (WR) {
        // step d stores point row d + 1
#pragma unroll
        for (int d = 0; d < DPW; ++d) issue_wload(d + 1, prew[d]);
    }
    // level k emits its last row (Lin - 1 - kR) at step Lin - 1 - kR + 2Rk;
    // it is stored one step later
    const int Q = a.Lin + R * k + 1;
    auto run = [&](auto bt) {
        for (int q = 0; q < Q; q += U) {
            static_for<0, U>([&](auto dc) {
                constexpr int d = decltype(dc)::value;
                step(q + d, pre[d % DP], bt, dc);
            });
        }
    };
    if (!PER && border_tile)
        run(std::true_type{});
    else
        run(std::false_type{});
}

// LDS layout of a band of radius R: sub-row stride S (at least the lane
// groups of a row plus one pad group on each side, odd so that the staging
// writes of consecutive threads spread over the banks), row stride C*S,
// planes of (H + 2R) rows in 3D, R + 1 slots per level.
struct LayoutR {
    int S, Wp, PSP;
};
inline LayoutR layout_r(int D, int R, int C, int W, int H) {
    LayoutR l;
    l.S = W / C + 2;
    if (l.S % 2 == 0) ++l.S;
    l.Wp = C * l.S;
    const int plane = D == 3 ? (H + 2 * R) * l.Wp : l.Wp;
    l.PSP = plane + (plane % 2 == 0 ? 1 : 0);
    return l;
}

// vc: variable coefficients; a band with the weight ring adds 2Rk + 2 slots
// of P rows
inline size_t ndr_lds_bytes(const Problem& p, const BandGeom& g, bool vc = false) {
    const LayoutR l = layout_r(p.ndim, p.radius, g.C, g.W, g.H);
    size_t n = (size_t)(g.k + 1) * (p.radius + 1) * l.PSP;
    const int npt = (g.H * g.W + g.NT - 1) / g.NT;
    if (ndr_weight_ring(vc, p.ndim, p.radius, npt))
        n += (size_t)(2 * p.radius * g.k + 2) * p.order * l.Wp;
    return n * p.elem_bytes();
}

inline ArgsNd make_args_r(const Problem& p, const BandGeom& g) {
    const int D = p.ndim, R = p.radius;
    ArgsNd a{};
    a.nz = (int)p.dims[0];
    a.ny = D == 3 ? (int)p.dims[1] : 1;
    a.nx = (int)p.dims[D - 1];
    a.k = g.k;
    a.W = g.W;
    a.H = g.H;
    a.Wv = g.Wv;
    a.Hv = g.Hv;
    a.Gx = g.W / g.C;
    const LayoutR l = layout_r(D, R, g.C, g.W, g.H);
    a.S = l.S;
    a.Wp = l.Wp;
    a.PSP = l.PSP;
    a.G = g.G;
    a.NT = g.NT;
    a.Lv = g.Lv;
    a.Lin = g.Lv + 2 * g.k * R;
    a.ntx = g.ntx;
    a.nseg = g.nseg;
    a.nty = g.nty;
    a.lanemap = g.lanemap;
    a.ix0 = a.iy0 = a.is0 = 0;
    a.ix1 = a.ntx;
    a.iy1 = a.nty;
    a.is1 = a.nseg;
    if (p.boundary != TVS_PERIODIC) {
        // the kernel's own test: a tile is interior when it reaches no fixed point
        auto range = [R](int n_tiles, int valid, int halo, int ext, int n, int* lo, int* hi) {
            *lo = n_tiles;
            *hi = 0;
            for (int t = 0; t < n_tiles; ++t) {
                const int org = t * valid - halo;
                if (org >= R && org + ext - 1 < n - R) {
                    *lo = std::min(*lo, t);
                    *hi = std::max(*hi, t + 1);
                }
            }
        };
        const int halo = g.k * R;
        range(a.ntx, a.Wv, halo, a.W, a.nx, &a.ix0, &a.ix1);
        range(a.nseg, a.Lv, halo, a.Lin, a.nz, &a.is0, &a.is1);
        if (D == 3) range(a.nty, a.Hv, halo, a.H, a.ny, &a.iy0, &a.iy1);
        if (a.ix1 <= a.ix0 || a.iy1 <= a.iy0 || a.is1 <= a.is0)
            a.ix0 = a.ix1 = a.iy0 = a.iy1 = a.is0 = a.is1 = 0;
    }
    return a;
}

template <typename T, int D, bool BOX, int R, bool VC>
hipError_t launch_ndr_impl(const Problem& p, const BandGeom& g, const T* in, T* out,
                           const Coeffs<T>& cf, const T* wts, hipStream_t st) {
    const ArgsNd a = make_args_r(p, g);
    const size_t lds = ndr_lds_bytes(p, g, VC);
    const int npt = (a.H * a.W + a.NT - 1) / a.NT;
    const bool per = p.boundary == TVS_PERIODIC;
    dim3 grid((unsigned)g.blocks()), block((unsigned)g.NT);
    hipError_t err = hipErrorInvalidValue;
    auto go = [&](auto kern) {
        static bool attr_set = false;  // per instantiation
        if (!attr_set) {
            (void)hipFuncSetAttribute((const void*)kern,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            attr_set = true;
        }
        hipLaunchKernelGGL(kern, grid, block, lds, st, in, out, a, cf, wts);
        err = hipGetLastError();
    };
#define TVS_NDR(PR, CC, N) go(tstp_ndr<T, D, BOX, R, PR, CC, N, VC>)
#define TVS_NDR_N(PR, CC)                          \
    do {                                           \
        if (npt <= 1) TVS_NDR(PR, CC, 1);          \
        else if (npt <= 2) TVS_NDR(PR, CC, 2);     \
        else if (npt <= 4) TVS_NDR(PR, CC, 4);     \
        else return hipErrorInvalidValue;          \
    } while (0)
    // 8 points per lane only for 2D constant weights (elsewhere the
    // running sums and weights of 8 points per lane exceed the registers)
#define TVS_NDR_C(PR)                                              \
    if (g.C == 4) {                                                \
        TVS_NDR_N(PR, 4);                                          \
    } else if constexpr (D == 2 && !VC) {                          \
        if (g.C == 8) TVS_NDR_N(PR, 8);                            \
        else return hipErrorInvalidValue;                          \
    } else {                                                       \
        return hipErrorInvalidValue;                               \
    }
    if (per) { TVS_NDR_C(true) } else { TVS_NDR_C(false) }
#undef TVS_NDR_C
#undef TVS_NDR_N
#undef TVS_NDR
    return err;
}

}  // namespace ndr
}  // namespace tvs
