// Longest common subsequence as a 1D Gauss-Seidel-like stencil (Section 3.4,
// "Longest common subsequence").
//
// The table lcs[x][y] (x = 1..m the time axis, y = 1..n the space axis) is
//   lcs[x][y] = lcs[x-1][y-1] + 1              if A[x] == B[y],
//             = max(lcs[x-1][y], lcs[x][y-1])  otherwise.
// A point needs the new value of its west neighbour and the previous row's
// values at y and y-1, so successive rows can run in successive lanes with a
// skew of one position per lane (Section 3.2's legality rule gives s >= 1
// here), and B acts as a coefficient that varies along the space axis.
//
// Tiling: rectangles of rows x tw columns (Section 3.4: LCS allows
// rectangle tiling), one wave per 64 rows.  Lane g holds row x0+g and, at step q,
// computes column y0+q-g.  Its north value is lane g-1's output of the
// previous step and its north-west value lane g-1's output of the step
// before (both through a DPP shift by one lane); B moves down the lanes the
// same way.  Lane 0 takes the top row and B from registers that hold 64
// steps' worth, one value per lane, rotated down one lane per step.  Before
// its first column a lane's output register holds its row's left boundary,
// which is exactly the north-west value its successor needs at its own first
// column.
//
// Tiles of one anti-diagonal I + J = d are independent and run in one
// launch; launch d+1 starts after launch d, so no workgroup ever waits for
// another.  The wavefront arrays of the paper are the caller's row (the
// bottom row of the tiles above, n+1 values) and column (the right column of
// the tiles to the left, m+1 values), updated in place: a tile reads its part
// of both at the start and overwrites it at the end.  The corner
// lcs[x0-1][y0-1] of tile (I, J) is the left-boundary value of the last row
// of tile (I-1, J); that tile saves it in corner[J] before overwriting the
// column (tile (0, J) gets it from the boundary row, saved before any tile
// runs).
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>

#include "kernels.hpp"

struct tvs_lcs {
    int64_t m = 0, n = 0;
    int tw = 1024;   // tile columns
    int rows = 256;  // tile rows: 64 per wave
    int nI = 0, nJ = 0;
    int32_t* corner = nullptr;
};

// Corner array of the allocation-free run (stencil_lcs_run_noalloc): one
// int32 per tile column, held by every device the library runs on until the
// process ends.  Host code never uses this name as an address; it takes the
// device's own address from hipGetSymbolAddress (noalloc_corner below).
constexpr int kLcsNoAllocCorners = 65536;
static __device__ __align__(256) int32_t scratch[kLcsNoAllocCorners];

namespace tvs {
namespace {

constexpr int kLcsPad = 192;  // row-buffer slack: 64 leading slots and a chunk past the last step

// Before the tiles: save the corners of the top tiles, and the two values of
// the results that no tile writes (lcs[0][n] and lcs[m][0]).
__global__ void lcs_init(int32_t* row, int32_t* col, int32_t* corner, int m, int n, int tw,
                         int nJ) {
    const int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J == 0) {
        const int32_t r0 = row[0], rn = row[n], cm = col[m];
        if (nJ > 0) corner[0] = r0;
        col[0] = rn;
        if (m >= 1) row[0] = cm;
    } else if (J < nJ) {
        corner[J] = row[J * tw];
    }
}

__device__ __forceinline__ int32_t lane_shift(int32_t x, int32_t first) {
    return dpp32<kDppWaveShr1>(first, x);  // lane i <- lane i-1; lane 0 <- first
}
// lane i <- lane i+1; lane 63 reads 0 (bound_ctrl), so the move needs no old
// value and the compiler no copy of it
__device__ __forceinline__ int32_t lane_rotate_down(int32_t x) {
    return __builtin_amdgcn_update_dpp(0, x, kDppWaveShl1, 0xF, 0xF, true);
}

// The tiles of anti-diagonal d, one workgroup of W = blockDim.x / 64 waves
// each: wave w holds rows x0 + 64w .. x0 + 64w + 63 and runs the one-wave
// pipeline below on its own step count q (lane j computes column q - j).
// Its lane 0 takes the row above from rowbuf[w]: the top boundary for wave
// 0, the bottom row of wave w-1 otherwise, which that wave's lane 63 emits
// (column q - 63 at its step q).  Waves advance in rounds of 64 steps with a
// barrier between rounds; wave w runs its chunk c in round c + 2w, when wave
// w-1 has emitted every column the chunk reads (they come from its chunks c
// and c+1).  Rows past the end of A (in the last band) act as a delay line:
// they copy their north value, so the last wave's lane 63 always emits the
// bottom row of the tile.  A register rotated down one lane per step gathers
// lane 63's outputs, stored once per chunk: to LDS for the next wave, to HBM
// for the last one.
__global__ __launch_bounds__(1024) void lcs_diag(const uint8_t* __restrict__ a,
                                                 const uint8_t* __restrict__ b, int32_t* row,
                                                 int32_t* col, int32_t* corner, int m, int n,
                                                 int tw, int nI, int nJ, int d) {
    extern __shared__ int32_t sm[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int W = (int)blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int I = max(0, d - (nJ - 1)) + (int)blockIdx.x;
    const int J = d - I;
    const int x0 = 1 + 64 * W * I;        // the tile's first row
    const int y0 = 1 + J * tw;            // and first column
    const int twt = min(tw, n - y0 + 1);  // columns of this tile
    const int S = tw + kLcsPad;           // row-buffer length; column c at index 64 + c
    int32_t* bv = sm;                     // B[y0+i] at i
    int32_t* rb = sm + S;                 // rowbuf[v] = rb + v * S
    for (int i = tid; i < S; i += 64 * W) {
        bv[i] = i < twt ? (int32_t)b[y0 - 1 + i] : -1;
        rb[i] = (i >= 64 && i - 64 < twt) ? row[y0 + i - 64] : 0;
    }
    const int x = x0 + 64 * w + lane;
    const bool vrow = x <= m;
    const int32_t ax = vrow ? (int32_t)a[x - 1] : -2;  // never equal to a B value
    const int32_t west0 = vrow ? col[x] : 0;           // lcs[x][y0-1]
    // lcs[x0+64w-1][y0-1]: the saved corner for wave 0, else the row above's
    // left boundary (a row of this tile, not yet overwritten)
    const int xa = x0 + 64 * w - 1;
    const int32_t cor = w == 0 ? corner[J] : (xa <= m ? col[xa] : 0);
    // a delay-line lane takes max(north, INT_MIN) = north at every step
    const int32_t cap = vrow ? INT32_MAX : INT32_MIN;
    const unsigned span = vrow ? (unsigned)twt : 0xffffffffu;
    const bool full_tile = x0 + 64 * W - 1 <= m;  // uniform
    __syncthreads();
    int32_t out = west0;                // this row's latest value
    int32_t nw = lane_shift(out, cor);  // lcs[x-1][y0-1] for the first column
    int32_t bq = -1;
    const int nch = (twt + 63 + 63) / 64;  // chunks: lane 63 emits column twt-1 at step twt+62
    const int32_t* src = rb + w * S + 64;
    int32_t* dst = w + 1 < W ? rb + (w + 1) * S + 1 : nullptr;  // column c at dst[63 + c]
    for (int round = 0; round < nch + 2 * (W - 1); ++round) {
        const int c = round - 2 * w;
        if (c >= 0 && c < nch) {
            const int q0 = 64 * c;
            // this chunk's row-above values and letters of B, one per lane;
            // lane 0 takes step mm's pair after mm rotations
            int32_t tin = src[q0 + lane], bin = bv[q0 + lane];
            int32_t obot = 0;  // lane 63's outputs of this chunk, oldest in lane 0
            // CHECK: lanes may be outside their column range at some step of
            // the chunk (the first chunk, and chunks reaching past the tile's
            // last column); in the others every lane computes at every step
            // FULL: every row of the tile exists (all but the last band), so
            // no lane is a delay line and the west value needs no cap
            auto chunk = [&](auto check, auto full) {
                static_for<0, 64>([&](auto mc) {
                    constexpr int mm = decltype(mc)::value;
                    // rotate first: the shifts below then consume tin and bin
                    const int32_t tnext = lane_rotate_down(tin);
                    const int32_t bnext = lane_rotate_down(bin);
                    const int32_t N = lane_shift(out, tin);  // lcs[x-1][y]
                    bq = lane_shift(bq, bin);                 // B[y]
                    tin = tnext;
                    bin = bnext;
                    const int32_t west = decltype(full)::value ? out : min(out, cap);
                    const int32_t f = bq == ax ? nw + 1 : max(N, west);
                    if constexpr (decltype(check)::value) {
                        const bool valid = (unsigned)(q0 + mm - lane) < span;
                        out = valid ? f : out;
                    } else {
                        out = f;
                    }
                    nw = N;
                    obot = dpp32<kDppWaveShl1>(out, obot);  // lane 63 <- its own output
                });
            };
            const bool inner = q0 >= 64 && q0 + 64 <= twt;
            if (full_tile) {
                if (inner) chunk(std::false_type{}, std::true_type{});
                else chunk(std::true_type{}, std::true_type{});
            } else {
                if (inner) chunk(std::false_type{}, std::false_type{});
                else chunk(std::true_type{}, std::false_type{});
            }
            // lane i holds column q0 + i - 63 of this wave's bottom row
            const int yc = q0 + lane - 63;
            if (dst) {
                dst[q0 + lane] = obot;
            } else if (yc >= 0 && yc < twt) {
                row[y0 + yc] = obot;
            }
        }
        __syncthreads();
    }
    if (vrow) col[x] = out;
    if (w == W - 1 && lane == 63 && I + 1 < nI) corner[J] = west0;  // lcs[x0+64W-1][y0-1]
}

// The device address of `scratch` on the current device, looked up once per
// device with that device current (each device holds its own copy).
int noalloc_corner(int32_t** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static int32_t* addr[kMaxDevices] = {};
    int dev = 0;
    TVS_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(TVS_E_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* ptr = nullptr;
        TVS_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return set_error(TVS_E_DEVICE, "no device address for the LCS scratch array");
        addr[dev] = (int32_t*)ptr;
    }
    *out = addr[dev];
    return TVS_OK;
}

}  // namespace

static size_t lcs_lds_bytes(int tw, int rows) {
    return (size_t)(1 + rows / 64) * (size_t)(tw + kLcsPad) * sizeof(int32_t);
}

static int parse_lcs_tuning(const char* t, int* tw, int* rows) {
    if (!t || !*t) return TVS_OK;
    std::string s(t);
    size_t pos = 0;
    while (pos < s.size()) {
        size_t end = s.find(',', pos);
        if (end == std::string::npos) end = s.size();
        const std::string kv = s.substr(pos, end - pos);
        pos = end + 1;
        if (kv.empty()) continue;
        const bool is_w = kv.compare(0, 2, "w=") == 0, is_r = kv.compare(0, 2, "r=") == 0;
        if (!is_w && !is_r) return set_error(TVS_E_INVALID, "unknown LCS tuning " + kv);
        char* e = nullptr;
        const long v = std::strtol(kv.c_str() + 2, &e, 10);
        if (!e || *e || v < 64 || v % 64 || v > (is_w ? 4096 : 1024))
            return set_error(TVS_E_INVALID, is_w ? "LCS tile width must be a multiple of 64 in 64..4096"
                                                 : "LCS tile rows must be a multiple of 64 in 64..1024");
        (is_w ? *tw : *rows) = (int)v;
    }
    return TVS_OK;
}

}  // namespace tvs

using namespace tvs;

extern "C" {

int stencil_lcs_plan(tvs_lcs** out, int64_t m, int64_t n, const char* tuning) {
    clear_error();
    if (!out) return set_error(TVS_E_INVALID, "out is NULL");
    // the kernels index rows and columns in 32 bits, up to a tile (at most
    // 1024 rows, 4096 columns) plus a pipeline's lag past the last one
    constexpr int64_t kMax = (int64_t)1 << 30;
    if (m < 0 || n < 0 || m > kMax || n > kMax)
        return set_error(TVS_E_SHAPE, "sequence lengths must lie in 0..2^30");
    // measured on 200000 x 200000 over widths 128..2048 and heights 64..1024:
    // 1024 x 256 best (1012 GCells/s; 512 x 256: 906, 1024 x 512: 921)
    int tw = 1024, rows = 256;
    int rc = parse_lcs_tuning(tuning, &tw, &rows);
    if (rc) return rc;
    if (lcs_lds_bytes(tw, rows) > 160 * 1024)
        return set_error(TVS_E_INVALID, "LCS tile too large for LDS: (rows/64 + 1) x (w + 192) "
                                        "int32 values must fit 160 KiB");
    tvs_lcs* p = new (std::nothrow) tvs_lcs();
    if (!p) return set_error(TVS_E_NOMEM, "out of host memory");
    p->m = m;
    p->n = n;
    p->tw = tw;
    p->rows = rows;
    p->nI = (int)((m + rows - 1) / rows);
    p->nJ = (int)((n + tw - 1) / tw);
    *out = p;
    return TVS_OK;
}

int stencil_lcs_tile_width(const tvs_lcs* p) { return p ? p->tw : TVS_E_INVALID; }
int stencil_lcs_tile_rows(const tvs_lcs* p) { return p ? p->rows : TVS_E_INVALID; }

}  // extern "C"

namespace tvs {

// The run's launches, with the corner array of at least max(1, nJ) int32.
static int lcs_enqueue(const tvs_lcs* p, const uint8_t* a, const uint8_t* b, int32_t* row,
                       int32_t* col, int32_t* corner, hipStream_t st) {
    const int m = (int)p->m, n = (int)p->n;
    const int nthreads = std::max(1, p->nJ);
    hipLaunchKernelGGL(lcs_init, dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0, st, row,
                       col, corner, m, n, p->tw, p->nJ);
    TVS_HIP_TRY(hipGetLastError());
    if (m == 0 || n == 0) return TVS_OK;
    const size_t lds = lcs_lds_bytes(p->tw, p->rows);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void*)lcs_diag, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr_set = true;
    }
    for (int d = 0; d < p->nI + p->nJ - 1; ++d) {
        const int ilo = std::max(0, d - (p->nJ - 1)), ihi = std::min(p->nI - 1, d);
        hipLaunchKernelGGL(lcs_diag, dim3((unsigned)(ihi - ilo + 1)), dim3(p->rows), lds, st, a, b, row,
                           col, corner, m, n, p->tw, p->nI, p->nJ, d);
    }
    TVS_HIP_TRY(hipGetLastError());
    return TVS_OK;
}

}  // namespace tvs

extern "C" {

int stencil_lcs_run(tvs_lcs* p, const uint8_t* a, const uint8_t* b, int32_t* row, int32_t* col,
                    void* stream) {
    clear_error();
    if (!p || !row || !col || (p->m > 0 && !a) || (p->n > 0 && !b))
        return set_error(TVS_E_INVALID, "NULL argument");
    if (!p->corner) {
        void* ptr = nullptr;
        if (hipMalloc(&ptr, (size_t)std::max(1, p->nJ) * sizeof(int32_t)) != hipSuccess)
            return set_error(TVS_E_NOMEM, "hipMalloc of the LCS corner array failed");
        p->corner = (int32_t*)ptr;
    }
    return lcs_enqueue(p, a, b, row, col, p->corner, (hipStream_t)stream);
}

int stencil_lcs_run_noalloc(const tvs_lcs* p, const uint8_t* a, const uint8_t* b, int32_t* row,
                            int32_t* col, void* stream) {
    clear_error();
    if (!p || !row || !col || (p->m > 0 && !a) || (p->n > 0 && !b))
        return set_error(TVS_E_INVALID, "NULL argument");
    if (p->nJ > kLcsNoAllocCorners)
        return set_error(TVS_E_SHAPE, "stencil_lcs_run_noalloc: ceil(n / w) tile columns exceed "
                                      "the 65536 entries of the static corner array");
    int32_t* corner = nullptr;
    int rc = noalloc_corner(&corner);
    if (rc) return rc;
    return lcs_enqueue(p, a, b, row, col, corner, (hipStream_t)stream);
}

int stencil_lcs_destroy(tvs_lcs* p) {
    clear_error();
    if (!p) return TVS_OK;
    if (p->corner) {
        (void)hipDeviceSynchronize();
        (void)hipFree(p->corner);
    }
    delete p;
    return TVS_OK;
}

}  // extern "C"
