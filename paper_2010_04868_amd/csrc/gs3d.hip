// Gauss-Seidel in 3D: in-place lexicographic sweeps (Section 3.4,
// "Gauss-Seidel stencils") pipelined over time along a hyperplane wavefront.
//
// A point (i, j, k) of a lexicographic sweep reads the new values of the
// neighbours that precede it in lexicographic order and the old values of
// the others.  With plane index pi = wi*i + wj*j + k -- weights (1, 1, 1) for
// the star, (4, 2, 1) for the box -- every preceding neighbour lies on a
// lower plane and every following one on a higher plane (the box's offsets
// (-1, b, c) give -4 + 2b + c <= -1; (0, -1, c) give -2 + c <= -1), at most
// D = 1 (star) or 7 (box) planes away.  So a sweep is exact when its planes
// are updated in increasing order, all points of one plane at once.
//
// Sweeps are pipelined the way the paper pipelines time steps (Section 3.2):
// K successive sweeps run together, sweep t+1 trailing sweep t by G = D + 1
// planes, so that one launch updates plane d of sweep t+1, plane d + G of
// sweep t, plane d + 2G of sweep t-1, ...  Sweep t+1 then reads new values
// (planes d-D .. d-1) that it wrote in earlier launches and old values
// (planes d+1 .. d+D) that sweep t finished in earlier launches and has not
// yet passed; the planes written in one launch are G apart, so no point is
// read and written by different threads of a launch.  The arithmetic of each
// point is the canonical chain, so the result is bit-identical to the naive
// sweep for every K.  A group of K sweeps takes planes + G (K - 1) launches;
// launch order alone orders the planes, so no workgroup waits for another.
//
// Storage: plane-major for the duration of a run.  A plane's points sit along
// a diagonal of the C-order grid (consecutive points n2-1 elements apart), so
// every neighbour read of a plane update would take a cache line of its own.
// The work area holds the grid as L[d][i][j] (k = d - wi*i - wj*j): the
// neighbour (i+a, j+b, k+c) of a point is at L[d + wi*a + wj*b + c][i+a][j+b],
// rows of neighbouring planes that consecutive threads (consecutive j) read
// at consecutive addresses.  Entries whose k falls outside the grid are never
// read.  The layout takes (wi + wj + 1) times the grid's memory plus the
// border planes: 3x for the star, 7x for the box.
#include <algorithm>

#include "kernels.hpp"

namespace tvs {
namespace {

struct Gs3dGeom {
    int n0, n1, n2;
    int wi, wj;
    int nplanes;  // d = 0 .. nplanes-1 (border points included)
};

Gs3dGeom gs3d_geom(const Problem& p) {
    Gs3dGeom g;
    g.n0 = (int)p.dims[0];
    g.n1 = (int)p.dims[1];
    g.n2 = (int)p.dims[2];
    const bool box = p.shape == TVS_BOX;
    g.wi = box ? 4 : 1;
    g.wj = box ? 2 : 1;
    g.nplanes = g.wi * (g.n0 - 1) + g.wj * (g.n1 - 1) + (g.n2 - 1) + 1;
    return g;
}

// Grid <-> plane-major layout; thread = one grid point (coalesced on the grid side).
template <typename T, bool IN>
__global__ __launch_bounds__(256) void gs3d_layout(T* grid, T* lay, Gs3dGeom g) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)g.n0 * g.n1 * g.n2;
    if (e >= total) return;
    const int k = (int)(e % g.n2);
    const int64_t r = e / g.n2;
    const int j = (int)(r % g.n1);
    const int i = (int)(r / g.n1);
    const int d = g.wi * i + g.wj * j + k;
    const int64_t at = ((int64_t)d * g.n0 + i) * g.n1 + j;
    if (IN)
        lay[at] = grid[e];
    else
        grid[e] = lay[at];
}

template <typename T, bool BOX>
__global__ __launch_bounds__(256) void gs3d_planes(T* lay, Gs3dGeom g, Coeffs<T> cf, int L,
                                                   int G, int dmin, int dmax, int jblocks) {
    using S = Stencil<3, BOX>;
    constexpr int WI = BOX ? 4 : 1, WJ = BOX ? 2 : 1;
    // blocks: sweep slot fastest (slots G planes apart share rows of the
    // planes between them, so they run together and meet in L2), then
    // column blocks; blockIdx.y is the row
    const int K = (int)gridDim.x / jblocks;
    const int slot = (int)blockIdx.x % K, jb = (int)blockIdx.x / K;
    const int d = dmin + L - G * slot;  // slot s: the s-th oldest sweep of the group
    if (d < dmin || d > dmax) return;   // uniform per workgroup
    const int i = 1 + (int)blockIdx.y;
    // row i of plane d holds the points with k = d - WI*i - WJ*j in 1..n2-2:
    // threads start at the first such j (ceil((d - WI*i - (n2-2)) / WJ), at least 1)
    const int num = d - WI * i - (g.n2 - 2);
    const int jlo = max(1, num <= 0 ? -((-num) / WJ) : (num + WJ - 1) / WJ);
    const int j = jlo + jb * 256 + (int)threadIdx.x;
    const int k = d - WI * i - WJ * j;
    if (j > g.n1 - 2 || k < 1 || k > g.n2 - 2) return;
    const int64_t rowp = g.n1, planep = (int64_t)g.n0 * g.n1;
    const int64_t at = ((int64_t)d * g.n0 + i) * g.n1 + j;
    T acc = 0;
    static_for<0, S::P>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int a = S::off(q, 0), b = S::off(q, 1), c = S::off(q, 2);
        constexpr int dd = WI * a + WJ * b + c;
        acc = term(acc, cf.c[q], lay[at + dd * planep + a * rowp + b], q == 0);
    });
    lay[at] = acc;
}

template <typename T>
hipError_t launch_gs3d_t(const Problem& p, T* lay, const Coeffs<T>& cf, int sweeps,
                         hipStream_t st) {
    const bool box = p.shape == TVS_BOX;
    const Gs3dGeom g = gs3d_geom(p);
    if (sweeps < 1 || sweeps > 65535 || g.n0 - 2 > 65535 || g.n0 < 3 || g.n1 < 3 || g.n2 < 3)
        return hipErrorInvalidValue;
    const int G = box ? 8 : 2;
    const int dmin = g.wi + g.wj + 1;  // interior planes
    const int dmax = g.wi * (g.n0 - 2) + g.wj * (g.n1 - 2) + (g.n2 - 2);
    // points per (plane, row): at most n2-2 (star) or ceil((n2-2)/2) (box), and at most n1-2
    const int jspan = std::min(g.n1 - 2, box ? (g.n2 - 2 + 1) / 2 : g.n2 - 2);
    const int jblocks = (jspan + 255) / 256;
    const dim3 grid((unsigned)(sweeps * jblocks), (unsigned)(g.n0 - 2));
    const int launches = (dmax - dmin + 1) + G * (sweeps - 1);
    for (int L = 0; L < launches; ++L) {
        if (box)
            hipLaunchKernelGGL((gs3d_planes<T, true>), grid, dim3(256), 0, st, lay, g, cf, L, G,
                               dmin, dmax, jblocks);
        else
            hipLaunchKernelGGL((gs3d_planes<T, false>), grid, dim3(256), 0, st, lay, g, cf, L, G,
                               dmin, dmax, jblocks);
    }
    return hipGetLastError();
}

template <typename T, bool IN>
hipError_t layout3_t(const Problem& p, T* grid, T* lay, hipStream_t st) {
    const Gs3dGeom g = gs3d_geom(p);
    const int64_t total = (int64_t)g.n0 * g.n1 * g.n2;
    hipLaunchKernelGGL((gs3d_layout<T, IN>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       st, grid, lay, g);
    return hipGetLastError();
}

}  // namespace

size_t gs3d_layout_bytes(const Problem& p) {
    const Gs3dGeom g = gs3d_geom(p);
    return (size_t)g.nplanes * (size_t)g.n0 * (size_t)g.n1 * p.elem_bytes();
}

// The layout lives in the work area after its 256-byte state block.
hipError_t gs3d_layout(const Problem& p, void* grid, void* work, bool in, hipStream_t st) {
    void* lay = (char*)work + 256;
    if (p.dtype == TVS_F64)
        return in ? layout3_t<double, true>(p, (double*)grid, (double*)lay, st)
                  : layout3_t<double, false>(p, (double*)grid, (double*)lay, st);
    return in ? layout3_t<float, true>(p, (float*)grid, (float*)lay, st)
              : layout3_t<float, false>(p, (float*)grid, (float*)lay, st);
}

hipError_t launch_gs3d(const Problem& p, void* work, const void* coeffs, int sweeps,
                       hipStream_t st) {
    void* lay = (char*)work + 256;
    if (p.dtype == TVS_F64)
        return launch_gs3d_t<double>(p, (double*)lay, *(const Coeffs<double>*)coeffs, sweeps, st);
    return launch_gs3d_t<float>(p, (float*)lay, *(const Coeffs<float>*)coeffs, sweeps, st);
}

}  // namespace tvs
