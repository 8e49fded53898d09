// Time-skewed temporal pipeline for 2D and 3D Jacobi stencils.
//
// Temporal vectorization applies to the outermost space loop only (Section
// 3.2, "High-dimensional Stencils"), so axis 0 is the stream axis and the
// other axes are tiled.  A workgroup owns one tile and a segment of the
// stream axis for a band of k time steps.  Its lanes are grouped by time
// level: lane group j (j = 1..k) holds level t0+j.  At every step all levels
// advance one stream position together, level j working s = 2 positions
// behind level j-1, so a vector of lanes holds points of k successive time
// levels at skewed stream positions -- the paper's input/output vectors --
// and no lane ever waits for a value of its own step (the legality
// condition s > max dx/dt of Section 3.2 is s >= 2 for radius 1).
//
// The values a level hands to the next are stored in LDS, one plane per
// level and stream position parity (Section 3.2: in higher dimensions the
// reorganized input vectors are stored for the following outer iterations).
// Within a plane row, element x of lane group g = x / C sits at
// (x mod C) * S + g + 1: same-position values of consecutive lanes are
// contiguous -- the transposed layout of Section 3.3.  The planes of one
// parity are consecutive, PSP elements apart, and S and PSP are padded so
// that the lanes' reads and writes and the staging accesses spread over the
// LDS banks (lds_layout.cpp).  One barrier per step separates the writers of
// one parity from the readers of the other.
//
// Level 0 is staged from HBM a few steps ahead; level k goes through its own
// LDS plane and is stored by all threads one step later, so loads and stores
// are coalesced and each grid value crosses HBM once per band of k steps.  Tiles overlap by k
// points per side on the tiled axes and at the segment ends (a trapezoid in
// time), so workgroups never wait for each other.
//
// Every level computes each point with the canonical operation order,
// carried as three running sums per point: the terms of the stencil row
// behind the point along the stream axis, at it, and ahead of it -- contiguous
// runs of the canonical order.  When all weights are equal the product of a
// value and the weight is computed once per value and used by every term
// that needs it; a product is the same rounded number wherever it is used,
// so this changes no bit.  The result is bit-identical to the naive sweep.
//
// Game of Life (LIFE, 2D box on 32-bit cells) runs the same pipeline with
// every weight one: the finished running sum is the 3 x 3 sum around the
// point, the point's own value is the centre value its lane read one step
// earlier, and the B2S23 rule maps the two to the new cell.
#pragma once

#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace tvs {
namespace nd {

struct ArgsNd {
    int nz, ny, nx;   // stream axis, axis 1 (3D only, else 1), last axis
    int k;
    int W, H;         // tile extents (halo included)
    int Wv, Hv;       // valid extents
    int S;            // LDS sub-row stride (elements); row stride is C*S
    int Wp;           // LDS row stride (elements)
    int PSP;          // LDS plane stride (elements); plane (level l, parity r)
                      // starts at (r * (k + 1) + l) * PSP
    int G, Gx, NT;    // lanes per level, lane groups per tile row, threads
    int Lv, Lin;
    int ntx, nty, nseg;
    int lanemap;
    // interior tile ranges [lo, hi) per axis: tiles that touch no fixed
    // border (all tiles under periodic boundaries)
    int ix0, ix1, iy0, iy1, is0, is1;
};

// Dispatch order of a band's tiles.  Tiles that touch a fixed border run the
// slower border path; dispatched first, they overlap the interior tiles
// instead of trailing them.  The interior tiles follow, spread so that each
// XCD takes a contiguous range of them (neighbouring tiles share halo data
// in its L2).  Maps block index blk to the tile's lexicographic index
// (stream segment, row, column); a bijection on [0, tiles).
__host__ __device__ inline int tile_order(int blk, const ArgsNd& a) {
    const int ntx = a.ntx, nty = a.nty;
    const int nix = a.ix1 - a.ix0, niy = a.iy1 - a.iy0, nis = a.is1 - a.is0;
    const int plane = ntx * nty;
    const int ni = nix * niy * nis;
    const int nb = plane * a.nseg - ni;
    auto lex = [&](int bs, int by, int bx) { return (bs * nty + by) * ntx + bx; };
    if (blk >= nb) {  // interior
        const int t = xcd_block(blk - nb, ni);
        const int r = t / nix;
        return lex(a.is0 + r / niy, a.iy0 + r % niy, a.ix0 + t % nix);
    }
    int r = blk;
    const int before = a.is0 * plane;  // whole planes before the interior segments
    if (r < before) return r;
    r -= before;
    const int per = plane - nix * niy;  // border tiles of a plane of an interior segment
    if (r < nis * per) {
        const int bs = a.is0 + r / per;
        int q = r % per;
        if (q < a.iy0 * ntx) return lex(bs, q / ntx, q % ntx);  // rows before
        q -= a.iy0 * ntx;
        const int m = ntx - nix;  // border tiles of an interior row
        if (q < niy * m) {
            const int qq = q % m;
            return lex(bs, a.iy0 + q / m, qq < a.ix0 ? qq : a.ix1 + (qq - a.ix0));
        }
        q -= niy * m;
        return lex(bs, a.iy1 + q / ntx, q % ntx);  // rows after
    }
    return lex(a.is1, 0, 0) + (r - nis * per);  // whole planes after
}

// One tile of one band.  Threads tid >= a.NT take part in the barriers only
// (AW: the block has exactly a.NT threads).  Returns after a final LDS
// barrier, so the caller may reuse the LDS.
template <typename T, int D, bool BOX, bool PER, int C, int NPT, bool UNI, bool AW = false,
          bool LIFE = false>
__device__ __forceinline__ void tstp_tile(const T* __restrict__ in, T* __restrict__ out,
                                          const ArgsNd& a, const Coeffs<T>& cf, int tile, T* lds,
                                          int tid) {
    static_assert(!LIFE || (D == 2 && BOX && !UNI && std::is_unsigned<T>::value),
                  "Life: 2D box neighbourhood on unsigned 32-bit arithmetic");
    using St = Stencil<D, BOX>;
    constexpr int gm_b = St::group_begin(-1), gm_e = St::group_end(-1);
    constexpr int g0_b = St::group_begin(0), g0_e = St::group_end(0);
    constexpr int gp_b = St::group_begin(1), gp_e = St::group_end(1);
    static_assert(gm_b == 0 && gm_e == g0_b && g0_e == gp_b && gp_e == St::P, "canonical groups");
    constexpr int R = D == 3 ? 3 : 1;  // plane rows a lane reads
    constexpr int MID = D == 3 ? 1 : 0;

    const bool worker = AW || tid < a.NT;
    const int k = a.k;
    const int S = a.S;
    const int Wp = a.Wp;
    int b = tile;
    const int bx = b % a.ntx;
    b /= a.ntx;
    const int by = b % a.nty;
    const int bs = b / a.nty;
    const int x_org = bx * a.Wv - k;
    const int y_org = D == 3 ? by * a.Hv - k : 0;
    const int z_org = bs * a.Lv - k;

    int j, g;
    if (a.lanemap == 0) {
        j = 1 + tid % k;
        g = tid / k;
    } else {
        j = 1 + tid / a.G;
        g = tid % a.G;
    }
    if (!worker) {  // idle thread: valid addresses, no stores
        j = 1;
        g = 0;
    }
    const int ly = D == 3 ? g / a.Gx : 0;  // lane's tile row (3D)
    const int gx = g - ly * a.Gx;          // lane group within the row
    const int lx = gx * C;                 // lane's first tile column

    // Dirichlet: does this tile touch a fixed border?  (uniform branch)
    bool border_tile = false;
    if (!PER) {
        border_tile = x_org <= 0 || x_org + a.W - 1 >= a.nx - 1 || z_org <= 0 ||
                      z_org + a.Lin - 1 >= a.nz - 1;
        if (D == 3) border_tile = border_tile || y_org <= 0 || y_org + a.H - 1 >= a.ny - 1;
    }
    const int gy_lane = y_org + ly;
    const bool y_border = D == 3 && !PER && (gy_lane == 0 || gy_lane == a.ny - 1);

    // LDS plane of time level l (0..k) and stream-position parity r
    auto plane = [&](int l, int r) -> T* { return lds + (r * (k + 1) + l) * a.PSP; };

    // zero the LDS planes once (pads stay zero; they only feed invalid points)
    if (worker)
        for (int e = tid; e < (k + 1) * 2 * a.PSP; e += a.NT) lds[e] = T(0);

    // Staging: thread handles elements e = tid + i*NT of a tile plane, both to
    // load level 0 from HBM into LDS and to store level k from LDS to HBM.
    // The LDS position of element (row yl, column xl) is the one the lanes use.
    // Global accesses go through per-plane buffer resources: a thread without
    // an element, or without a valid output, gets an out-of-range offset, and
    // a row outside the segment gets an empty resource, so every step issues
    // the same loads and stores (no branch around them).
    const int PS = a.H * a.W;
    int st_lds[NPT];
    uint32_t ld_off[NPT], st_off[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int e = tid + i * a.NT;
        st_lds[i] = -1;
        ld_off[i] = st_off[i] = kBufOOB;
        if (worker && e < PS) {
            const int yl = D == 3 ? e / a.W : 0;
            const int xl = e - yl * a.W;
            const int ox = x_org + xl, oy = y_org + yl;
            int gxx = PER ? (int)wrap_idx(ox, a.nx) : (int)clamp_idx(ox, a.nx);
            int gyy = D == 3 ? (PER ? (int)wrap_idx(oy, a.ny) : (int)clamp_idx(oy, a.ny)) : 0;
            st_lds[i] = (D == 3 ? (yl + 1) * Wp : 0) + (xl % C) * S + xl / C + 1;
            ld_off[i] = (uint32_t)(gyy * a.nx + gxx) * (uint32_t)sizeof(T);
            const bool valid = xl >= k && xl < a.W - k && ox < a.nx &&
                               (D != 3 || (yl >= k && yl < a.H - k && oy < a.ny));
            if (valid) st_off[i] = (uint32_t)(oy * a.nx + ox) * (uint32_t)sizeof(T);
        }
    }
    // Row addresses in 32-bit scalar arithmetic: a plane is below 2 GiB, so
    // row * plane_bytes is one 32 x 32 -> 64-bit product.
    const uint32_t plane_bytes = (uint32_t)a.ny * (uint32_t)a.nx * (uint32_t)sizeof(T);
    auto row_ptr = [&](const T* base, int row) {
        return (const T*)((const char*)base + (uint64_t)(uint32_t)row * plane_bytes);
    };
    // periodic: the row of the next load, wrapped incrementally (loads are
    // issued for q = 0, 1, 2, ... in order)
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
    // par: parity of q, known at compile time in the unrolled step loop
    auto store_input = [&](int q, const T* v, int par) {
        if (q >= a.Lin) return;
        T* pl = plane(0, par);
#pragma unroll
        for (int i = 0; i < NPT; ++i)
            if (st_lds[i] >= 0) pl[st_lds[i]] = v[i];
    };
    // level k emitted tile row q-1-2k at step q-1 into its plane; write it out
    auto store_output = [&](int q, int par) {
        const int row = q - 1 - 2 * k;
        const int gz = z_org + row;
        const bool ok = row >= k && row < a.Lin - k && gz < a.nz;
        const T* pl = plane(k, par ^ 1);
        const auto rs = buf_rsrc(row_ptr(out, ok ? gz : 0), ok ? plane_bytes : 0u);
#pragma unroll
        for (int i = 0; i < NPT; ++i) buf_store<T>(rs, st_off[i], pl[st_lds[i] < 0 ? 0 : st_lds[i]]);
    };

    // Running sums of a lane's points, two per point.  At a step of parity r,
    // Acc[r] lacks only the terms of the stencil row ahead (it becomes this
    // step's output) and Acc[r^1] lacks the centre and ahead rows (it gains
    // the centre row in place); Acc[r] then starts the sums of the new row.
    // The roles swap with the parity, so no value is copied.
    T Acc[2][C];
    // Dirichlet: a fixed border point has the same value at every level, so
    // its level-j value is level j-1's value at the same point -- the centre
    // value this lane read one step earlier (stream row p-1).  Keeping those
    // raw values avoids a global load (and its wait) in the step.  Life needs
    // the same value (the cell's own state) at every point.
    T prevc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) Acc[0][c] = Acc[1][c] = prevc[c] = T(0);
    const T cu = cf.c[0];  // the common weight when UNI

    const int row_off = D == 3 ? ly * Wp : 0;  // padded row ly holds tile row ly-1
    // level-0 planes are loaded DP steps before they enter LDS: the wait for a
    // load then also covers the stores issued before it, which are DP steps old
    constexpr int DP = 4;
    T pre[DP][NPT];
#pragma unroll
    for (int d = 0; d < DP; ++d)
#pragma unroll
        for (int i = 0; i < NPT; ++i) pre[d][i] = T(0);

    // BT: this tile touches a fixed Dirichlet border (uniform per workgroup)
    auto step = [&](int q, T* pr, auto bt, auto dc) {
        constexpr bool BT = !PER && decltype(bt)::value;
        constexpr int par = decltype(dc)::value & 1;  // q & 1
        store_input(q, pr, par);
        issue_load(q + DP, pr);
        store_output(q, par);
        const int p = q - 2 * j + 1;  // stream position of the level-(j-1) plane read now
        // Interior tiles compute at every step, also outside the level's
        // stream range [0, Lin): such steps read rows not (or no longer)
        // produced and store garbage rows, but a valid output row r of a level
        // reads only rows r-1..r+1 of the level below, which are valid, and
        // its running sum is assigned afresh two steps before it is stored;
        // garbage only ever reaches rows outside the trapezoid, which are
        // never stored to HBM.  This keeps divergent branches out of the step.
        if (!BT || (p >= 0 && p < a.Lin)) {
            const T* src = plane(j - 1, par ^ 1) + row_off;
            // Shared products (equal weights) in interior tiles only: a border
            // tile multiplies every term by its weight -- with equal weights the
            // same rounded product -- so that v keeps the raw values, which
            // are also the fixed border values of the next step (prevc).
            constexpr bool SHARE = UNI && !BT && !LIFE;
            // v[r][i]: plane row ly-1+r, tile column lx-1+i (multiplied by the
            // common weight when SHARE)
            T v[R][C + 2];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T* rs = src + r * Wp;
#pragma unroll
                for (int i = 0; i < C + 2; ++i) {
                    const bool need = BOX || r == MID || (i >= 1 && i <= C);
                    if (!need) continue;
                    const int pos = i == 0 ? (C - 1) * S + gx : i <= C ? (i - 1) * S + gx + 1 : gx + 2;
                    v[r][i] = rs[pos];
                }
            }
            if constexpr (SHARE) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int i = 0; i < C + 2; ++i) {
                        const bool need = BOX || r == MID || (i >= 1 && i <= C);
                        if (need) v[r][i] = cu * v[r][i];
                    }
            }
            auto val = [&](auto qc, int c) -> T {
                constexpr int q2 = decltype(qc)::value;
                if constexpr (D == 3)
                    return v[1 + St::off(q2, 1)][1 + c + St::off(q2, 2)];
                else
                    return v[0][1 + c + St::off(q2, 1)];
            };
            // one canonical term: weight * value, or the shared product
            // (Life: the value itself)
            auto add = [&](T acc, auto qc, int c, bool first) -> T {
                constexpr int q2 = decltype(qc)::value;
                const T prod = SHARE || LIFE ? val(qc, c) : cf.c[q2] * val(qc, c);
                return first ? prod : acc + prod;
            };
            const int gz_out = z_org + p - 1;
            const bool z_border = !PER && (gz_out == 0 || gz_out == a.nz - 1);
            const bool emit = worker && (!BT || p >= 1);
            T* dst = plane(j, par) + (D == 3 ? row_off + Wp : 0) + gx + 1;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T f = Acc[par][c];
                static_for<gp_b, gp_e>([&](auto qc) { f = add(f, qc, c, false); });
                T m = Acc[par ^ 1][c];
                static_for<g0_b, g0_e>([&](auto qc) { m = add(m, qc, c, false); });
                T s = T(0);
                static_for<gm_b, gm_e>([&](auto qc) {
                    s = add(s, qc, c, decltype(qc)::value == gm_b);
                });
                Acc[par ^ 1][c] = m;
                Acc[par][c] = s;
                if constexpr (LIFE) {
                    // B2S23: born with 2 live neighbours, survives with 2 or 3
                    const T nbr = f - prevc[c];
                    f = (nbr == 2u || (prevc[c] != 0u && nbr == 3u)) ? T(1) : T(0);
                }
                if (emit) dst[c * S] = f;
                if constexpr (BT) {
                    // a fixed border point keeps its input value at every level:
                    // its lane overwrites the stored sum (a second, masked LDS
                    // store, so that the sum itself is computed unconditionally)
                    const int gxc = x_org + lx + c;
                    const bool fixed = z_border || y_border || gxc == 0 || gxc == a.nx - 1;
                    if (emit && fixed) dst[c * S] = prevc[c];
                }
                if constexpr (BT || LIFE) prevc[c] = v[MID][1 + c];
            }
        }
        lds_barrier();
    };

    lds_barrier();  // LDS zeroed
#pragma unroll
    for (int d = 0; d < DP; ++d) issue_load(d, pre[d]);
    // level k emits its last row at step Lin+k-1; it is stored one step later.
    // The loop body is DP steps, so that the prefetch slot and the plane
    // parity of every step are compile-time constants.  Whole groups run:
    // the extra steps load and store nothing (empty resources) and compute
    // nothing (p >= Lin for every level).
    static_assert(DP % 2 == 0, "even unroll: the parity of a step is its slot's");
    const int Q = a.Lin + k + 1;
    auto run = [&](auto bt) {
        for (int q = 0; q < Q; q += DP) {
            static_for<0, DP>([&](auto dc) {
                constexpr int d = decltype(dc)::value;
                step(q + d, pre[d], bt, dc);
            });
        }
    };
    // interior tiles, the vast majority, carry no border code at all
    if (!PER && border_tile)
        run(std::true_type{});
    else
        run(std::false_type{});
}

template <typename T, int D, bool BOX, bool PER, int C, int NPT, bool UNI, bool LIFE = false>
__global__ __launch_bounds__(512) void tstp_nd(const T* __restrict__ in, T* __restrict__ out,
                                               ArgsNd a, Coeffs<T> cf) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    tstp_tile<T, D, BOX, PER, C, NPT, UNI, true, LIFE>(in, out, a, cf, tile_order(blockIdx.x, a),
                                                 reinterpret_cast<T*>(smem_raw), threadIdx.x);
}

// Paddings S (sub-row stride), Wp = C * S (row stride) and PSP (plane
// stride) of a band geometry, in elements; see lds_layout.cpp.
struct LdsLayout {
    int S, Wp, PSP;
};
LdsLayout lds_layout(int D, bool box, int eb, int C, int W, int H, int k, int lanemap, int NT,
                     int G);

inline LdsLayout lds_layout(const Problem& p, const BandGeom& g) {
    return lds_layout(p.ndim, p.shape == TVS_BOX, (int)p.elem_bytes(), g.C, g.W, g.H, g.k,
                      g.lanemap, g.NT, g.G);
}

// Kernel arguments of a band (host side).
inline ArgsNd make_args(const Problem& p, const BandGeom& g) {
    const int D = p.ndim;
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
    const LdsLayout lay = lds_layout(p, g);
    a.S = lay.S;
    a.Wp = lay.Wp;
    a.PSP = lay.PSP;
    a.G = g.G;
    a.NT = g.NT;
    a.Lv = g.Lv;
    a.Lin = g.Lv + 2 * g.k;
    a.ntx = g.ntx;
    a.nseg = g.nseg;
    a.nty = g.nty;
    a.lanemap = g.lanemap;
    // interior ranges, by the same test the kernel applies (border_tile)
    a.ix0 = a.iy0 = a.is0 = 0;
    a.ix1 = a.ntx;
    a.iy1 = a.nty;
    a.is1 = a.nseg;
    if (p.boundary != TVS_PERIODIC) {
        auto range = [](int n_tiles, int valid, int k, int ext, int n, int* lo, int* hi) {
            *lo = n_tiles;
            *hi = 0;
            for (int t = 0; t < n_tiles; ++t) {
                const int org = t * valid - k;
                if (org > 0 && org + ext - 1 < n - 1) {
                    *lo = std::min(*lo, t);
                    *hi = std::max(*hi, t + 1);
                }
            }
        };
        range(a.ntx, a.Wv, a.k, a.W, a.nx, &a.ix0, &a.ix1);
        range(a.nseg, a.Lv, a.k, a.Lin, a.nz, &a.is0, &a.is1);
        if (D == 3) range(a.nty, a.Hv, a.k, a.H, a.ny, &a.iy0, &a.iy1);
        if (a.ix1 <= a.ix0 || a.iy1 <= a.iy0 || a.is1 <= a.is0)
            a.ix0 = a.ix1 = a.iy0 = a.iy1 = a.is0 = a.is1 = 0;  // no interior tile
    }
    return a;
}

// LIFE: Game of Life bands (box, periodic or Dirichlet, never uniform)
template <typename T, int D, bool LIFE = false>
hipError_t launch_nd_impl(const Problem& p, const BandGeom& g, const T* in, T* out,
                          const Coeffs<T>& cf, bool uniform, hipStream_t st) {
    const ArgsNd a = make_args(p, g);
    const size_t lds = (size_t)(g.k + 1) * 2 * a.PSP * sizeof(T);
    const int npt = (a.H * a.W + a.NT - 1) / a.NT;  // plane elements per thread
    const bool box = p.shape == TVS_BOX, per = p.boundary == TVS_PERIODIC;
    dim3 grid((unsigned)g.blocks()), block((unsigned)g.NT);
    hipError_t err = hipErrorInvalidValue;
    auto go = [&](auto kern) {
        static bool attr_set = false;  // per instantiation
        if (!attr_set) {
            (void)hipFuncSetAttribute((const void*)kern,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            attr_set = true;
        }
        hipLaunchKernelGGL(kern, grid, block, lds, st, in, out, a, cf);
        err = hipGetLastError();
    };
#define TVS_ND(B, PR, CC, N, U) go(tstp_nd<T, D, B, PR, CC, N, U, LIFE>)
#define TVS_ND_U(B, PR, CC, N)                                         \
    do {                                                               \
        if constexpr (LIFE) TVS_ND(B, PR, CC, N, false);               \
        else if (uniform) TVS_ND(B, PR, CC, N, true);                  \
        else TVS_ND(B, PR, CC, N, false);                              \
    } while (0)
#define TVS_ND_N(B, PR, CC)                               \
    do {                                                  \
        if (npt <= 1) TVS_ND_U(B, PR, CC, 1);             \
        else if (npt <= 2) TVS_ND_U(B, PR, CC, 2);        \
        else if (npt <= 4) TVS_ND_U(B, PR, CC, 4);        \
        else return hipErrorInvalidValue;                 \
    } while (0)
#define TVS_ND_C(B, PR)                      \
    switch (g.C) {                           \
        case 4: TVS_ND_N(B, PR, 4); break;   \
        case 8: TVS_ND_N(B, PR, 8); break;   \
        case 16: TVS_ND_N(B, PR, 16); break; \
        default: return hipErrorInvalidValue; \
    }
    if constexpr (LIFE) {
        if (!box) return hipErrorInvalidValue;
        if (per) { TVS_ND_C(true, true) } else { TVS_ND_C(true, false) }
    } else if (box) {
        if (per) { TVS_ND_C(true, true) } else { TVS_ND_C(true, false) }
    } else {
        if (per) { TVS_ND_C(false, true) } else { TVS_ND_C(false, false) }
    }
#undef TVS_ND_C
#undef TVS_ND_N
#undef TVS_ND_U
#undef TVS_ND
    return err;
}

}  // namespace nd

// LDS bytes a band of this geometry needs (same formula as the launcher).
inline size_t tstp_nd_lds_bytes(const Problem& p, const BandGeom& g) {
    return (size_t)(g.k + 1) * 2 * nd::lds_layout(p, g).PSP * p.elem_bytes();
}

hipError_t launch_nd_f64_2d(const Problem&, const BandGeom&, const double*, double*,
                            const Coeffs<double>&, bool, hipStream_t);
hipError_t launch_nd_f64_3d(const Problem&, const BandGeom&, const double*, double*,
                            const Coeffs<double>&, bool, hipStream_t);
hipError_t launch_nd_f32_2d(const Problem&, const BandGeom&, const float*, float*,
                            const Coeffs<float>&, bool, hipStream_t);
hipError_t launch_nd_f32_3d(const Problem&, const BandGeom&, const float*, float*,
                            const Coeffs<float>&, bool, hipStream_t);
hipError_t launch_nd_life_2d(const Problem&, const BandGeom&, const uint32_t*, uint32_t*,
                             hipStream_t);

}  // namespace tvs
