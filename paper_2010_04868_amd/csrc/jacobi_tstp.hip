// Time-skewed temporal pipeline (TSTP) for Jacobi stencils.
//
// The paper's central idea (Section 3.2, "Algorithm"): a vector holds points
// of successive time levels, t_{i+1} - t_i = 1, placed s apart along the
// space axis that is swept, so that one pass over the grid advances it by
// as many steps as the vector has lanes.  On gfx950 the vector is a group of
// lanes:
//
//   1D (tstp1d): a pipeline of PL lanes (a 16-lane DPP row or a whole
//   64-lane wave) sweeps a segment.  Lane j holds level j+1.  Each step a
//   lane receives the level-j value one position further along from lane
//   j-1 by a single DPP shift -- the rotate-and-blend of Algorithm 3 in one
//   cross-lane move, with the fresh level-0 value entering lane 0 through the
//   DPP "old" operand -- finishes one level-(j+1) point and hands it on.
//   Level-0 values arrive as a coalesced "bottom vector" once per PL steps
//   and the last lane's outputs are the top of the band (Section 3.2, top and
//   bottom vectors).
//
//   2D/3D (tstp_nd): temporal vectorization applies to the outermost space
//   loop only (Section 3.2, "High-dimensional Stencils"), so axis 0 is the
//   stream axis.  Lane group j of a workgroup holds level j; at every step
//   all levels advance one stream position together, level j working s = 2
//   positions behind level j-1 (the legality condition s > max dx/dt of
//   Section 3.2 gives s >= 2 for radius 1).  The values a level hands to the
//   next are kept in LDS planes, one per level and stream position -- the
//   "transposed layout" of Section 3.3, where same-time values of
//   consecutive input vectors sit contiguously -- so the inner-axis
//   neighbours are read from LDS and each grid value crosses HBM once per
//   band of k steps.
//
// Tiles overlap by k points per side on the non-stream axes and on the
// stream-axis segment ends (a trapezoid in time), so workgroups never wait
// for each other.  Every level computes each point with the canonical
// operation order, carried in three running sums per point (the terms of
// the stencil rows behind, at and ahead of the point along the stream axis,
// which are contiguous in canonical order), so the result is bit-identical
// to the naive sweep.
#include "kernels.hpp"

namespace tvs {
namespace {

// ---------------------------------------------------------------------------
// 1D
// ---------------------------------------------------------------------------
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

template <typename T, bool PER, int PL>
__global__ __launch_bounds__(256) void tstp1d(const T* __restrict__ in, T* __restrict__ out,
                                              Args1d a, Coeffs<T> cf) {
    const int lane = threadIdx.x & 63;
    const int j = lane % PL;  // lane j computes level j+1
    const int64_t seg = ((int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * (64 / PL) +
                        lane / PL;
    if (seg >= a.nseg) return;  // whole pipelines only (PL divides 64)
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

// ---------------------------------------------------------------------------
// 2D / 3D
// ---------------------------------------------------------------------------
struct ArgsNd {
    int nz, ny, nx;   // stream axis, axis 1 (3D only, else 1), last axis
    int k;
    int W, H;         // tile extents (halo included)
    int Wv, Hv;       // valid extents
    int Wp;           // LDS row stride (elements)
    int PSP;          // LDS plane stride (elements)
    int G, Gx, NT;    // lanes per level, lane groups per tile row, threads
    int Lv, Lin;
    int ntx, nty;
    int lanemap;
};

template <typename T, int D, bool BOX, bool PER, int C>
__global__ __launch_bounds__(512) void tstp_nd(const T* __restrict__ in, T* __restrict__ out,
                                               ArgsNd a, Coeffs<T> cf) {
    using S = Stencil<D, BOX>;
    constexpr int gm_b = S::group_begin(-1), gm_e = S::group_end(-1);
    constexpr int g0_b = S::group_begin(0), g0_e = S::group_end(0);
    constexpr int gp_b = S::group_begin(1), gp_e = S::group_end(1);
    static_assert(gm_b == 0 && gm_e == g0_b && g0_e == gp_b && gp_e == S::P, "canonical groups");
    constexpr int R = D == 3 ? 3 : 1;  // plane rows a lane reads
    constexpr int MID = D == 3 ? 1 : 0;

    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);

    const int tid = threadIdx.x;
    const int k = a.k;
    int b = blockIdx.x;
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
    const int ly = D == 3 ? g / a.Gx : 0;  // lane's tile row (3D)
    const int lx = (g % a.Gx) * C;         // lane's first tile column

    // Dirichlet: does this tile touch a fixed border?  (uniform branch)
    bool border_tile = false;
    if (!PER) {
        border_tile = x_org <= 0 || x_org + a.W - 1 >= a.nx - 1 || z_org <= 0 ||
                      z_org + a.Lin - 1 >= a.nz - 1;
        if (D == 3) border_tile = border_tile || y_org <= 0 || y_org + a.H - 1 >= a.ny - 1;
    }
    const int gy_lane = y_org + ly;
    const bool y_border = D == 3 && !PER && (gy_lane == 0 || gy_lane == a.ny - 1);

    // zero the LDS planes once (pads stay zero; they only feed invalid points)
    for (int e = tid; e < k * 2 * a.PSP; e += a.NT) lds[e] = T(0);

    // input staging: thread loads elements e = tid + i*NT of each input plane
    const int PS = a.H * a.W;
    int in_lds[C];
    int64_t in_g[C];
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const int e = tid + i * a.NT;
        in_lds[i] = -1;
        in_g[i] = 0;
        if (e < PS) {
            const int yl = D == 3 ? e / a.W : 0;
            const int xl = e - yl * a.W;
            int gx = x_org + xl, gyy = y_org + yl;
            gx = PER ? (int)wrap_idx(gx, a.nx) : (int)clamp_idx(gx, a.nx);
            if (D == 3) gyy = PER ? (int)wrap_idx(gyy, a.ny) : (int)clamp_idx(gyy, a.ny);
            in_lds[i] = (D == 3 ? (yl + 1) * a.Wp : 0) + xl + 1;
            in_g[i] = (int64_t)gyy * a.nx + gx;
        }
    }
    const int64_t plane_elems = (int64_t)a.ny * a.nx;
    auto issue_load = [&](int q, T* dst) {
        if (q >= a.Lin) return;
        int64_t gz = z_org + q;
        gz = PER ? wrap_idx(gz, a.nz) : clamp_idx(gz, a.nz);
        const T* src = in + gz * plane_elems;
#pragma unroll
        for (int i = 0; i < C; ++i)
            if (in_lds[i] >= 0) dst[i] = src[in_g[i]];
    };
    auto store_input = [&](int q, const T* v) {
        if (q >= a.Lin) return;
        T* pl = lds + (q & 1) * a.PSP;  // level 0, slot q&1
#pragma unroll
        for (int i = 0; i < C; ++i)
            if (in_lds[i] >= 0) pl[in_lds[i]] = v[i];
    };

    T Sacc[C], Macc[C], prevC[C];
#pragma unroll
    for (int c = 0; c < C; ++c) Sacc[c] = Macc[c] = prevC[c] = T(0);

    const int lane_off = (D == 3 ? ly * a.Wp : 0) + lx;  // (ly-1)+1 row, (lx-1)+1 column
    T pre0[C], pre1[C];
#pragma unroll
    for (int i = 0; i < C; ++i) pre0[i] = pre1[i] = T(0);

    auto step = [&](int q, T* pre) {
        store_input(q, pre);
        issue_load(q + 2, pre);
        const int p = q - 2 * j + 1;  // stream position of the level-(j-1) plane read now
        if (p >= 0 && p < a.Lin) {
            const T* src = lds + ((j - 1) * 2 + ((q - 1) & 1)) * a.PSP + lane_off;
            T v[R][C + 2];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int i = 0; i < C + 2; ++i) {
                    const bool need = BOX || r == MID || (i >= 1 && i <= C);
                    if (need) v[r][i] = src[r * a.Wp + i];
                }
            auto val = [&](auto qc, int c) -> T {
                constexpr int q2 = decltype(qc)::value;
                if constexpr (D == 3)
                    return v[1 + S::off(q2, 1)][1 + c + S::off(q2, 2)];
                else
                    return v[0][1 + c + S::off(q2, 1)];
            };
            const int gz_out = z_org + p - 1;
            const bool z_border = !PER && (gz_out == 0 || gz_out == a.nz - 1);
            T outv[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T f = Macc[c];
                static_for<gp_b, gp_e>([&](auto qc) {
                    f = term(f, cf.c[decltype(qc)::value], val(qc, c), false);
                });
                T m = Sacc[c];
                static_for<g0_b, g0_e>([&](auto qc) {
                    m = term(m, cf.c[decltype(qc)::value], val(qc, c), false);
                });
                T s = T(0);
                static_for<gm_b, gm_e>([&](auto qc) {
                    constexpr int q2 = decltype(qc)::value;
                    s = term(s, cf.c[q2], val(qc, c), q2 == gm_b);
                });
                if (border_tile) {
                    const int gx = x_org + lx + c;
                    if (z_border || y_border || gx == 0 || gx == a.nx - 1) f = prevC[c];
                }
                outv[c] = f;
                Macc[c] = m;
                Sacc[c] = s;
                prevC[c] = v[MID][1 + c];
            }
            if (p >= 1) {
                if (j < k) {
                    T* dst = lds + (j * 2 + (q & 1)) * a.PSP + lane_off + (D == 3 ? a.Wp : 0) + 1;
#pragma unroll
                    for (int c = 0; c < C; ++c) dst[c] = outv[c];
                } else {
                    const int row = p - 1;
                    const bool row_ok = row >= k && row < a.Lin - k && gz_out < a.nz &&
                                        (D != 3 || (ly >= k && ly < a.H - k && gy_lane < a.ny));
                    if (row_ok) {
                        T* o = out + ((int64_t)gz_out * a.ny + (D == 3 ? gy_lane : 0)) * a.nx;
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            const int xl = lx + c;
                            const int gx = x_org + xl;
                            if (xl >= k && xl < a.W - k && gx < a.nx) o[gx] = outv[c];
                        }
                    }
                }
            }
        }
        __syncthreads();
    };

    __syncthreads();  // LDS zeroed
    issue_load(0, pre0);
    issue_load(1, pre1);
    const int Q = a.Lin + k;
    for (int q = 0; q < Q; q += 2) {
        step(q, pre0);
        if (q + 1 < Q) step(q + 1, pre1);
    }
}

template <typename T, int D, bool BOX, bool PER>
hipError_t launch_nd(const Problem& p, const BandGeom& g, const T* in, T* out,
                     const Coeffs<T>& cf, hipStream_t st) {
    ArgsNd a{};
    a.nz = (int)p.dims[0];
    a.ny = D == 3 ? (int)p.dims[1] : 1;
    a.nx = (int)p.dims[D - 1];
    a.k = g.k;
    a.W = g.W;
    a.H = g.H;
    a.Wv = g.Wv;
    a.Hv = g.Hv;
    a.Wp = g.W + 2;
    a.PSP = (D == 3 ? (g.H + 2) * a.Wp : a.Wp);
    a.PSP += (a.PSP % 2 == 0) ? 1 : 0;  // odd plane stride spreads levels over banks
    a.G = g.G;
    a.Gx = g.W / g.C;
    a.NT = g.NT;
    a.Lv = g.Lv;
    a.Lin = g.Lv + 2 * g.k;
    a.ntx = g.ntx;
    a.nty = g.nty;
    a.lanemap = g.lanemap;
    const size_t lds = (size_t)g.k * 2 * a.PSP * sizeof(T);
    dim3 grid((unsigned)g.blocks()), block((unsigned)g.NT);
    switch (g.C) {
#define TVS_C(CC)                                                                              \
    case CC:                                                                                   \
        hipLaunchKernelGGL((tstp_nd<T, D, BOX, PER, CC>), grid, block, lds, st, in, out, a, cf); \
        break;
        TVS_C(1)
        TVS_C(2)
        TVS_C(4)
        TVS_C(8)
        TVS_C(16)
#undef TVS_C
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool PER>
hipError_t launch_1d(const Problem& p, const BandGeom& g, const T* in, T* out,
                     const Coeffs<T>& cf, hipStream_t st) {
    Args1d a{};
    a.n = p.dims[0];
    a.k = g.k;
    a.Lv = g.Lv;
    a.nseg = (a.n + g.Lv - 1) / g.Lv;
    const int pipes_per_block = 4 * (64 / g.pl);
    dim3 grid((unsigned)((a.nseg + pipes_per_block - 1) / pipes_per_block)), block(256);
    if (g.pl == 16)
        hipLaunchKernelGGL((tstp1d<T, PER, 16>), grid, block, 0, st, in, out, a, cf);
    else
        hipLaunchKernelGGL((tstp1d<T, PER, 64>), grid, block, 0, st, in, out, a, cf);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_band_t(const Problem& p, const BandGeom& g, const T* in, T* out,
                         const Coeffs<T>& cf, hipStream_t st) {
    const bool per = p.boundary == TVS_PERIODIC, box = p.shape == TVS_BOX;
    if (p.ndim == 1) return per ? launch_1d<T, true>(p, g, in, out, cf, st)
                                : launch_1d<T, false>(p, g, in, out, cf, st);
    if (p.ndim == 2) {
        if (box) return per ? launch_nd<T, 2, true, true>(p, g, in, out, cf, st)
                            : launch_nd<T, 2, true, false>(p, g, in, out, cf, st);
        return per ? launch_nd<T, 2, false, true>(p, g, in, out, cf, st)
                   : launch_nd<T, 2, false, false>(p, g, in, out, cf, st);
    }
    if (box) return per ? launch_nd<T, 3, true, true>(p, g, in, out, cf, st)
                        : launch_nd<T, 3, true, false>(p, g, in, out, cf, st);
    return per ? launch_nd<T, 3, false, true>(p, g, in, out, cf, st)
               : launch_nd<T, 3, false, false>(p, g, in, out, cf, st);
}

}  // namespace

bool tstp_supported(const Problem& p) {
    return p.dependence == TVS_JACOBI && p.radius == 1 && p.ndim >= 1 && p.ndim <= 3;
}

bool band_geometry(const Problem& p, const Schedule& s, int k, BandGeom* g) {
    BandGeom r;
    r.k = k;
    r.lanemap = s.lanemap;
    const size_t eb = p.elem_bytes();
    if (k < 1) return false;
    if (p.ndim == 1) {
        r.pl = s.pl == 16 ? 16 : 64;
        if (k > r.pl) return false;
        r.Lv = s.l > 0 ? s.l : 256;
        r.nseg = (int)((p.dims[0] + r.Lv - 1) / r.Lv);
        r.NT = 256;
        *g = r;
        return true;
    }
    r.C = s.c;
    if (r.C != 1 && r.C != 2 && r.C != 4 && r.C != 8 && r.C != 16) return false;
    r.W = s.w;
    if (r.W <= 2 * k || r.W % r.C) return false;
    r.Wv = r.W - 2 * k;
    if (p.ndim == 3) {
        r.H = s.h;
        if (r.H <= 2 * k) return false;
        r.Hv = r.H - 2 * k;
    } else {
        r.H = 1;
        r.Hv = 1;
    }
    r.G = r.H * r.W / r.C;
    r.NT = k * r.G;
    if (r.NT > 512) return false;
    // every thread must stage at most C input values per plane
    if ((int64_t)r.H * r.W > (int64_t)r.NT * r.C) return false;
    r.Lv = s.l > 0 ? s.l : 256;
    const int nstream = (int)p.dims[0];
    const int nxa = (int)p.dims[p.ndim - 1];
    r.ntx = (nxa + r.Wv - 1) / r.Wv;
    r.nty = p.ndim == 3 ? ((int)p.dims[1] + r.Hv - 1) / r.Hv : 1;
    r.nseg = (nstream + r.Lv - 1) / r.Lv;
    int Wp = r.W + 2;
    int PSP = p.ndim == 3 ? (r.H + 2) * Wp : Wp;
    PSP += PSP % 2 == 0 ? 1 : 0;
    r.lds_bytes = (size_t)k * 2 * PSP * eb;
    if (r.lds_bytes > 160 * 1024) return false;
    *g = r;
    return true;
}

hipError_t launch_tstp_band(const Problem& p, const BandGeom& g, const void* in, void* out,
                            const void* coeffs, hipStream_t st) {
    if (p.dtype == TVS_F64)
        return launch_band_t<double>(p, g, (const double*)in, (double*)out,
                                     *(const Coeffs<double>*)coeffs, st);
    return launch_band_t<float>(p, g, (const float*)in, (float*)out,
                                *(const Coeffs<float>*)coeffs, st);
}

}  // namespace tvs
