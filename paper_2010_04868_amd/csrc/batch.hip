// Batched launches: many Jacobi grids of uneven shapes and step counts
// advance together.
//
// The grids of one kernel variant (precision, dimension, shape, boundary,
// equal weights, points per lane) run together.  Every grid keeps the
// schedule its plan was tuned to (depth, tile shape, segment length, lane
// map); its bands are cut into tiles, and the work list holds every tile of
// every band of every grid in round-major order (band b of every grid before
// band b + 1 of any).  Band b reads what band b - 1 wrote and overwrites what
// it read.  Two ways to run a group:
//
//   * round launches (the default): one launch per round b over the round's
//     slice of the work list; the kernel boundary is the only
//     synchronization, so there are no waits between workgroups;
//   * one persistent launch (TVS_BATCH_PERSISTENT=1): workgroups take items
//     from an atomic ticket, and a tile of band b of grid g waits until all
//     tiles of the grid's earlier bands are done (a per-grid counter of
//     finished tiles).  Every wait points to an earlier ticket, held by a
//     workgroup that is running and never waits for a later one, so the
//     launch drains for any number of workgroups; the waits are bounded
//     anyway, and on expiry the launch records a status word and stops
//     waiting.  Each tile needs an agent-scope acquire before it reads and a
//     release after it writes; on a device whose XCDs have separate L2
//     caches those invalidate and write back a whole L2, once per tile,
//     which makes this form several times slower than round launches, whose
//     kernel boundaries pay the same once per round.
//
// The launch sequence of a batch layout that repeats is captured once in a
// hipGraph and replayed.
//
// Each tile runs the same tile body as a single-grid band, with the same
// canonical per-point arithmetic, so every grid's result is bit-identical
// to advancing it alone.
#include <algorithm>
#include <cstdlib>
#include <tuple>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "api_internal.hpp"
#include "plan.hpp"
#include "tstp1d.hpp"
#include "tstp_nd.hpp"

namespace tvs {
namespace {

constexpr int kBatchC = 4;    // nD points per lane of the batch's own schedules
constexpr int kBatchNPT = 4;  // nD: staging values per thread (any k >= C/4)
constexpr long long kBatchSpinLimit = 1ll << 22;  // ~seconds: far beyond any band
constexpr size_t kBatchLds = 160 * 1024;          // dynamic LDS of a persistent nD launch

struct BatchItem {
    unsigned int g;     // grid within the group
    unsigned int b;     // band
    unsigned int t;     // tile of the band
    unsigned int need;  // tiles of the grid's bands before b (all done before this one)
};

template <typename T>
struct GridNd {
    T* buf[2];
    nd::ArgsNd band[2];  // [0] full bands, [1] last band
    int nbands;
    int tiles[2];
    Coeffs<T> cf;
};

template <typename T>
struct Grid1d {
    T* buf[2];
    d1::Args1d band[2];
    int nbands;
    int tiles[2];
    Coeffs<T> cf;
};

// Layout of a group's synchronization words in device memory.
// Per-grid counters of finished tiles, one per cache line: the workgroups
// that poll a grid's counter and the tiles that bump it then share that line
// with no other grid's traffic.
constexpr int kDoneStride = 32;  // ints: 128 bytes
struct SyncWords {
    int ticket;
    int pad[63];   // the per-grid counters start on their own cache line
    int done[1];   // [ngrids * kDoneStride], grid g's counter at done[g * kDoneStride]
};

__global__ void batch_reset(int* sync, int ngrids) {
    auto* s = reinterpret_cast<SyncWords*>(sync);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) s->ticket = 0;
    for (int g = i; g < ngrids; g += gridDim.x * blockDim.x) s->done[g * kDoneStride] = 0;
}

// Take the next item and wait for the bands it depends on.  Called by wave 0
// only, every lane (no lane-dependent branch: the ticket is a scalar).
// Returns the item index (>= nitems: no more work).
__device__ __forceinline__ int take_item(const BatchItem* items, int nitems, SyncWords* s,
                                         int* status) {
    const int lane = threadIdx.x & 63;
    const int mine = atomicAdd(&s->ticket, lane == 0 ? 1 : 0);
    const int it = __builtin_amdgcn_readfirstlane(mine);
    if (it < nitems) {
        const unsigned g = items[it].g, need = items[it].need;
        const int* done = &s->done[g * kDoneStride];
        long long spins = 0;
        while ((unsigned)__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               need) {
            // the status word lives in host memory: reading it at every poll
            // from hundreds of waiting workgroups floods the host link and
            // slowed whole launches several-fold, so it is read every 256 polls
            if ((spins & 255) == 0 &&
                __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0)
                break;
            if (++spins > kBatchSpinLimit) {
                __hip_atomic_store(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    return it;
}

// After a tile: its stores are made visible device-wide by every thread,
// then one count per tile.
__device__ __forceinline__ void finish_item(SyncWords* s, unsigned g, int wave) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave == 0) {
        const int lane = threadIdx.x & 63;
        __hip_atomic_fetch_add(&s->done[g * kDoneStride], lane == 0 ? 1 : 0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Tiles of a batch form every product with its own weight (the single-grid
// kernel's shared products for equal weights give the same bits; the batch
// kernels skip that variant to halve their instantiations).
// The item slot that wave 0 hands to the other waves sits in dynamic LDS at
// byte offset slot_off, past every member's tile planes (a static __shared__
// variable would count against the 160 KiB the tile planes may take).
template <typename T, int D, bool BOX, bool PER, int C>
__global__ __launch_bounds__(512) void batch_persistent_nd(const GridNd<T>* grids,
                                                           const BatchItem* items, int nitems,
                                                           int* sync, int* status,
                                                           unsigned slot_off) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    int* s_item = reinterpret_cast<int*>(smem_raw + slot_off);
    auto* s = reinterpret_cast<SyncWords*>(sync);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (;;) {
        if (wave == 0) {
            const int it = take_item(items, nitems, s, status);
            *s_item = it;
        }
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(*s_item);
        if (it >= nitems) break;
        // the earlier bands' stores (other workgroups, other XCDs) are visible
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const BatchItem w = items[it];
        const GridNd<T>& gr = grids[w.g];
        const int which = (int)w.b == gr.nbands - 1 ? 1 : 0;
        nd::tstp_tile<T, D, BOX, PER, C, kBatchNPT, false>(
            gr.buf[w.b & 1], gr.buf[(w.b + 1) & 1], gr.band[which], gr.cf, (int)w.t,
            reinterpret_cast<T*>(smem_raw), threadIdx.x);
        finish_item(s, w.g, wave);  // also orders s_item's next write after every read
    }
}

// Round launches: block i runs item first + i of round `round`.
template <typename T, int D, bool BOX, bool PER, bool UNI, int C>
__global__ __launch_bounds__(512) void batch_round_nd(const GridNd<T>* grids,
                                                      const BatchItem* items, int round) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const BatchItem w = items[blockIdx.x];
    const GridNd<T>& gr = grids[w.g];
    const int which = round == gr.nbands - 1 ? 1 : 0;
    nd::tstp_tile<T, D, BOX, PER, C, kBatchNPT, UNI>(
        gr.buf[round & 1], gr.buf[(round + 1) & 1], gr.band[which], gr.cf, (int)w.t,
        reinterpret_cast<T*>(smem_raw), threadIdx.x);
}

template <typename T, bool PER>
__global__ __launch_bounds__(256) void batch_round_1d(const Grid1d<T>* grids,
                                                      const BatchItem* items, int round) {
    const BatchItem w = items[blockIdx.x];
    const Grid1d<T>& gr = grids[w.g];
    const int which = round == gr.nbands - 1 ? 1 : 0;
    d1::tstp1d_tile<T, PER, 64>(gr.buf[round & 1], gr.buf[(round + 1) & 1], gr.band[which],
                                gr.cf, (int)w.t, threadIdx.x);
}

template <typename T, bool PER>
__global__ __launch_bounds__(256) void batch_persistent_1d(const Grid1d<T>* grids,
                                                           const BatchItem* items, int nitems,
                                                           int* sync, int* status) {
    __shared__ int s_item;
    auto* s = reinterpret_cast<SyncWords*>(sync);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (;;) {
        if (wave == 0) {
            const int it = take_item(items, nitems, s, status);
            s_item = it;
        }
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= nitems) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const BatchItem w = items[it];
        const Grid1d<T>& gr = grids[w.g];
        const int which = (int)w.b == gr.nbands - 1 ? 1 : 0;
        d1::tstp1d_tile<T, PER, 64>(gr.buf[w.b & 1], gr.buf[(w.b + 1) & 1], gr.band[which],
                                    gr.cf, (int)w.t, threadIdx.x);
        finish_item(s, w.g, wave);
    }
}

template <typename T>
__global__ void copy_back(const T* __restrict__ src, T* __restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Variant {
    int dtype, ndim, shape, boundary, uniform, c;
    bool operator<(const Variant& o) const {
        return std::tie(dtype, ndim, shape, boundary, uniform, c) <
               std::tie(o.dtype, o.ndim, o.shape, o.boundary, o.uniform, o.c);
    }
};

bool persistent_mode() {
    const char* env = std::getenv("TVS_BATCH_PERSISTENT");
    return env && env[0] == '1';
}

struct Member {
    tvs_plan* plan;
    void* grid;
    const double* coeffs;
    int64_t T;
    Schedule sched;
};

// The batch's own schedule for a grid whose plan has no time-skewed one
// (plain or untuned): 4 points per lane, moderate depth.
Schedule batch_schedule(const Problem& p) {
    Schedule s;
    s.method = TVS_METHOD_TSTP;
    s.c = kBatchC;
    s.lanemap = 0;
    if (p.ndim == 1) {
        s.pl = 64;
        s.k = 64;
        s.l = (int)std::max<int64_t>(128, std::min<int64_t>(1024, p.dims[0] / 512));
    } else if (p.ndim == 2) {
        s.k = 8;
        s.w = 256;
        s.l = 128;
        while (s.w > 32 && s.w - 2 * s.k > 2 * p.dims[1]) s.w /= 2;
        if (s.w <= 2 * s.k) s.k = std::max(1, s.w / 4);
    } else {
        s.k = 2;
        s.w = 64;
        s.h = 16;
        s.l = 64;
        while (s.w > 16 && s.w - 2 * s.k > 2 * p.dims[2]) s.w /= 2;
        while (s.h > 8 && s.h - 2 * s.k > 2 * p.dims[1]) s.h /= 2;
    }
    return s;
}

// Whether a schedule runs every band of T steps in the batch kernels: its
// full bands and its last, shallower one (a lane group stages at most four
// plane values per step, so few levels of many points per lane may not fit).
bool batch_fits(const Problem& p, const Schedule& s, int64_t T) {
    if (p.ndim > 1 && s.c != 4 && s.c != 8) return false;
    const int kfull = (int)std::max<int64_t>(1, std::min<int64_t>(s.k, T));
    const int64_t nbands = (T + kfull - 1) / kfull;
    const int klast = (int)std::max<int64_t>(1, T - (nbands - 1) * kfull);
    BandGeom gf, gl;
    if (!band_geometry(p, s, kfull, &gf) || !band_geometry(p, s, klast, &gl)) return false;
    // the persistent launch keeps 16 bytes of LDS past the tile planes
    return p.ndim == 1 || std::max(gf.lds_bytes, gl.lds_bytes) + 32 <= kBatchLds;
}

// The schedule a member runs: its plan's (tuned) time-skewed schedule when
// the batch kernels can take it, else the batch's own (4 points per lane,
// which fits a band of any depth).  In 1D the batch pipelines are 64 lanes
// wide.
Schedule member_schedule(const Problem& p, const Schedule& plan_s, int64_t T) {
    if (plan_s.method == TVS_METHOD_TSTP) {
        Schedule s = plan_s;
        if (p.ndim == 1) {
            s.pl = 64;
            s.k = std::min(64, s.k);
        }
        if (batch_fits(p, s, T)) return s;
    }
    return batch_schedule(p);
}

template <typename T>
void fill_coeffs_t(const Problem& p, const double* c, Coeffs<T>* out) {
    for (int q = 0; q < kMaxPoints; ++q) out->c[q] = q < p.order ? (T)c[q] : T(0);
}

// Build the device descriptors and item list for one variant group; returns
// the LDS bytes the launch needs.
template <typename T>
int build_group(const std::vector<Member>& ms, int ndim, std::vector<GridNd<T>>* gnd,
                std::vector<Grid1d<T>>* g1d, std::vector<BatchItem>* items,
                std::vector<int>* round_begin, std::vector<int>* odd, size_t* lds_out) {
    size_t lds = 0;
    std::vector<std::vector<int>> tiles_per_band(ms.size());
    std::vector<int> nb(ms.size());
    for (size_t i = 0; i < ms.size(); ++i) {
        const Problem& p = ms[i].plan->prob;
        const Schedule& s = ms[i].sched;
        const int kfull = (int)std::min<int64_t>(s.k, ms[i].T);
        const int nbands = (int)((ms[i].T + kfull - 1) / kfull);
        const int klast = (int)(ms[i].T - (int64_t)(nbands - 1) * kfull);
        BandGeom gf, gl;
        if (!band_geometry(p, s, kfull, &gf) || !band_geometry(p, s, klast, &gl))
            return set_error(TVS_E_UNSUPPORTED, "batch tile shape does not fit a member grid");
        nb[i] = nbands;
        if (ndim == 1) {
            Grid1d<T> d{};
            d.buf[0] = (T*)ms[i].grid;
            d.buf[1] = (T*)ms[i].plan->scratch;
            for (int w = 0; w < 2; ++w) {
                const BandGeom& g = w ? gl : gf;
                d.band[w].n = p.dims[0];
                d.band[w].k = g.k;
                d.band[w].Lv = g.Lv;
                d.band[w].nseg = (p.dims[0] + g.Lv - 1) / g.Lv;
                d.tiles[w] = (int)((d.band[w].nseg + 3) / 4);
            }
            d.nbands = nbands;
            fill_coeffs_t(p, ms[i].coeffs, &d.cf);
            g1d->push_back(d);
            tiles_per_band[i].assign(nbands, d.tiles[0]);
            tiles_per_band[i][nbands - 1] = d.tiles[1];
        } else {
            GridNd<T> d{};
            d.buf[0] = (T*)ms[i].grid;
            d.buf[1] = (T*)ms[i].plan->scratch;
            d.band[0] = nd::make_args(p, gf);
            d.band[1] = nd::make_args(p, gl);
            d.tiles[0] = (int)gf.blocks();
            d.tiles[1] = (int)gl.blocks();
            d.nbands = nbands;
            fill_coeffs_t(p, ms[i].coeffs, &d.cf);
            lds = std::max(lds, std::max(tstp_nd_lds_bytes(p, gf), tstp_nd_lds_bytes(p, gl)));
            gnd->push_back(d);
            tiles_per_band[i].assign(nbands, d.tiles[0]);
            tiles_per_band[i][nbands - 1] = d.tiles[1];
        }
        if (nbands % 2) odd->push_back((int)i);
    }
    // round-major order: band b of every grid that has one, then band b + 1
    int maxb = 0;
    for (int v : nb) maxb = std::max(maxb, v);
    std::vector<unsigned> before(ms.size(), 0);  // tiles of the bands already listed
    for (int b = 0; b < maxb; ++b) {
        round_begin->push_back((int)items->size());
        for (size_t i = 0; i < ms.size(); ++i)
            if (b < nb[i]) {
                for (int t = 0; t < tiles_per_band[i][b]; ++t)
                    items->push_back(BatchItem{(unsigned)i, (unsigned)b, (unsigned)t, before[i]});
                before[i] += (unsigned)tiles_per_band[i][b];
            }
    }
    round_begin->push_back((int)items->size());
    *lds_out = lds;
    return TVS_OK;
}

// One group, prepared on the host.  Its work list ([items | grids | sync
// words]) is built as a host image and then uploaded either into memory the
// group owns (synchronously, before any stream work, so that the launches
// can be captured in a graph) or into caller-provided buffers
// (asynchronously).
struct GroupLaunch {
    Variant v;
    void* dev = nullptr;  // [items | grids | sync words]
    bool owned = false;   // dev was allocated for this group
    std::vector<unsigned char> image;
    size_t lds = 0;
    int nitems = 0, ngrids = 0;
    std::vector<int> round_begin;  // item offset of each round, plus the end
    size_t off_grids = 0, off_sync = 0;
    std::vector<std::pair<const void*, void*>> copies;  // odd band count: scratch -> grid
    std::vector<int64_t> copy_elems;
};

template <typename T>
int prepare_group(const Variant& v, const std::vector<Member>& ms, GroupLaunch* gl) {
    std::vector<GridNd<T>> gnd;
    std::vector<Grid1d<T>> g1d;
    std::vector<BatchItem> items;
    std::vector<int> odd;
    size_t lds = 0;
    gl->v = v;
    int rc = build_group<T>(ms, v.ndim, &gnd, &g1d, &items, &gl->round_begin, &odd, &lds);
    if (rc) return rc;
    gl->lds = lds;
    if (items.empty()) return TVS_OK;
    gl->nitems = (int)items.size();
    gl->ngrids = (int)ms.size();
    gl->off_grids = (items.size() * sizeof(BatchItem) + 255) & ~(size_t)255;
    const size_t grid_bytes =
        v.ndim == 1 ? g1d.size() * sizeof(Grid1d<T>) : gnd.size() * sizeof(GridNd<T>);
    gl->off_sync = (gl->off_grids + grid_bytes + 255) & ~(size_t)255;
    const size_t total = gl->off_sync + sizeof(SyncWords) + ms.size() * kDoneStride * sizeof(int);
    std::vector<unsigned char>& host = gl->image;
    host.assign(total, 0);
    std::memcpy(host.data(), items.data(), items.size() * sizeof(BatchItem));
    if (v.ndim == 1) std::memcpy(host.data() + gl->off_grids, g1d.data(), grid_bytes);
    else std::memcpy(host.data() + gl->off_grids, gnd.data(), grid_bytes);
    for (int i : odd) {
        gl->copies.emplace_back(ms[i].plan->scratch, ms[i].grid);
        gl->copy_elems.push_back(ms[i].plan->prob.elems());
    }
    return TVS_OK;
}

// Pinned status word shared by every persistent batch launch of the process:
// 0, or 1 once a launch's bounded wait expired (results of that batch are
// invalid).  Reported and cleared by the next stencil_batch_run.
int* batch_status_host() {
    static int* host = nullptr;
    static std::once_flag once;
    std::call_once(once, [] {
        void* h = nullptr;
        if (hipHostMalloc(&h, sizeof(int), hipHostMallocMapped | hipHostMallocCoherent) ==
            hipSuccess) {
            host = (int*)h;
            *host = 0;
        }
    });
    return host;
}

// Persistent workgroups of a kernel: as many as are resident at once on the
// device, but no more than there are items.
int persistent_blocks(const void* kern, int threads, size_t lds, int nitems) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return std::max(1, std::min(nitems, per_cu * std::max(1, cus)));
}

template <typename T>
int launch_rounds(const GroupLaunch& gl, hipStream_t st) {
    const Variant& v = gl.v;
    const int rounds = (int)gl.round_begin.size() - 1;
    for (int b = 0; b < rounds; ++b) {
        const int n = gl.round_begin[b + 1] - gl.round_begin[b];
        if (n <= 0) continue;
        auto* ditems = (const BatchItem*)gl.dev + gl.round_begin[b];
        if (v.ndim == 1) {
            auto* dg = (const Grid1d<T>*)((char*)gl.dev + gl.off_grids);
            if (v.boundary == TVS_PERIODIC)
                hipLaunchKernelGGL((batch_round_1d<T, true>), dim3(n), dim3(256), 0, st, dg, ditems, b);
            else
                hipLaunchKernelGGL((batch_round_1d<T, false>), dim3(n), dim3(256), 0, st, dg, ditems, b);
        } else {
            auto* dg = (const GridNd<T>*)((char*)gl.dev + gl.off_grids);
            const bool box = v.shape == TVS_BOX, per = v.boundary == TVS_PERIODIC, uni = v.uniform;
            const size_t lds = gl.lds;
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(n), dim3(512), lds, st, dg, ditems, b);
            };
#define TVS_R(DD, B, PR, U, CC) go(batch_round_nd<T, DD, B, PR, U, CC>)
#define TVS_RC(DD, B, PR, U)                                              \
    switch (v.c) {                                                        \
        case 4: TVS_R(DD, B, PR, U, 4); break;                            \
        case 8: TVS_R(DD, B, PR, U, 8); break;                            \
        default: return set_error(TVS_E_UNSUPPORTED, "batch lane width"); \
    }
#define TVS_RU(DD, B, PR)                                                 \
    if (uni) { TVS_RC(DD, B, PR, true) } else { TVS_RC(DD, B, PR, false) }
#define TVS_R3(DD)                                                        \
    if (box) {                                                            \
        if (per) { TVS_RU(DD, true, true) } else { TVS_RU(DD, true, false) }   \
    } else {                                                              \
        if (per) { TVS_RU(DD, false, true) } else { TVS_RU(DD, false, false) } \
    }
            if (v.ndim == 2) { TVS_R3(2) } else { TVS_R3(3) }
#undef TVS_R3
#undef TVS_RU
#undef TVS_RC
#undef TVS_R
        }
        TVS_HIP_TRY(hipGetLastError());
    }
    return TVS_OK;
}

template <typename T>
int launch_group(const GroupLaunch& gl, hipStream_t st) {
    if (!gl.dev || gl.image.empty() || gl.nitems == 0) return TVS_OK;
    const Variant& v = gl.v;
    if (!persistent_mode()) {
        int rc = launch_rounds<T>(gl, st);
        if (rc) return rc;
        for (size_t i = 0; i < gl.copies.size(); ++i) {
            const int64_t n = gl.copy_elems[i];
            hipLaunchKernelGGL(copy_back<T>, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)),
                               dim3(256), 0, st, (const T*)gl.copies[i].first,
                               (T*)gl.copies[i].second, n);
            TVS_HIP_TRY(hipGetLastError());
        }
        return TVS_OK;
    }
    int* host_status = batch_status_host();
    int* status = nullptr;
    if (!host_status || hipHostGetDevicePointer((void**)&status, host_status, 0) != hipSuccess)
        return set_error(TVS_E_DEVICE, "batch status word unavailable");
    int* sync = (int*)((char*)gl.dev + gl.off_sync);
    const auto* ditems = (const BatchItem*)gl.dev;
    hipLaunchKernelGGL(batch_reset, dim3((unsigned)std::max(1, (gl.ngrids + 255) / 256)),
                       dim3(256), 0, st, sync, gl.ngrids);
    TVS_HIP_TRY(hipGetLastError());
    if (v.ndim == 1) {
        auto* dg = (const Grid1d<T>*)((char*)gl.dev + gl.off_grids);
        auto go = [&](auto kern) {
            const int blocks = persistent_blocks((const void*)kern, 256, 0, gl.nitems);
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, st, dg, ditems, gl.nitems, sync,
                               status);
        };
        if (v.boundary == TVS_PERIODIC) go(batch_persistent_1d<T, true>);
        else go(batch_persistent_1d<T, false>);
    } else {
        auto* dg = (const GridNd<T>*)((char*)gl.dev + gl.off_grids);
        const bool box = v.shape == TVS_BOX, per = v.boundary == TVS_PERIODIC;
        const unsigned slot_off = (unsigned)((gl.lds + 15) & ~(size_t)15);
        const size_t lds = slot_off + 16;
        if (lds > kBatchLds) return set_error(TVS_E_UNSUPPORTED, "batch tile planes exceed LDS");
        auto go = [&](auto kern) {
            const int blocks = persistent_blocks((const void*)kern, 512, lds, gl.nitems);
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(512), lds, st, dg, ditems, gl.nitems,
                               sync, status, slot_off);
        };
#define TVS_B(DD, B, PR, CC) go(batch_persistent_nd<T, DD, B, PR, CC>)
#define TVS_BC(DD, B, PR)                                                 \
    switch (v.c) {                                                        \
        case 4: TVS_B(DD, B, PR, 4); break;                               \
        case 8: TVS_B(DD, B, PR, 8); break;                               \
        default: return set_error(TVS_E_UNSUPPORTED, "batch lane width"); \
    }
#define TVS_B3(DD)                                                                  \
    if (box) {                                                                      \
        if (per) { TVS_BC(DD, true, true) } else { TVS_BC(DD, true, false) }        \
    } else {                                                                        \
        if (per) { TVS_BC(DD, false, true) } else { TVS_BC(DD, false, false) }      \
    }
        if (v.ndim == 2) { TVS_B3(2) } else { TVS_B3(3) }
#undef TVS_B3
#undef TVS_BC
#undef TVS_B
    }
    TVS_HIP_TRY(hipGetLastError());
    for (size_t i = 0; i < gl.copies.size(); ++i) {
        const int64_t n = gl.copy_elems[i];
        hipLaunchKernelGGL(copy_back<T>, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)),
                           dim3(256), 0, st, (const T*)gl.copies[i].first, (T*)gl.copies[i].second, n);
        TVS_HIP_TRY(hipGetLastError());
    }
    return TVS_OK;
}

template <typename T>
void set_lds_attributes() {
    static std::once_flag once;
    std::call_once(once, [] {
        auto set = [](auto kern) {
            (void)hipFuncSetAttribute((const void*)kern,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        };
        static_for<0, 2>([&](auto dc) {
            constexpr int DD = decltype(dc)::value + 2;
            static_for<0, 4>([&](auto fc) {
                constexpr int f = decltype(fc)::value;
                constexpr bool B = f & 1, PR = (f >> 1) & 1;
                set(batch_persistent_nd<T, DD, B, PR, 4>);
                set(batch_persistent_nd<T, DD, B, PR, 8>);
                set(batch_round_nd<T, DD, B, PR, true, 4>);
                set(batch_round_nd<T, DD, B, PR, true, 8>);
                set(batch_round_nd<T, DD, B, PR, false, 4>);
                set(batch_round_nd<T, DD, B, PR, false, 8>);
            });
        });
    });
}

struct BatchPlan {
    std::vector<GroupLaunch> groups;
    std::vector<std::pair<tvs_plan*, int>> gs;  // Gauss-Seidel members (plan, index)
};

void free_batch(BatchPlan* bp) {
    for (auto& g : bp->groups)
        if (g.dev && g.owned) (void)hipFree(g.dev);
    bp->groups.clear();
}

// Upload the work lists of a prepared batch.  Without ext: one allocation per
// group, synchronous copies.  With ext: all lists packed into ext's pinned
// host staging and device buffer (grown if needed), one asynchronous copy on
// st; the caller keeps ext alive and unused by other work until the batch's
// launches have run.
int upload_batch(BatchPlan* bp, BatchBuffers* ext, hipStream_t st) {
    if (!ext) {
        for (auto& g : bp->groups) {
            if (g.image.empty()) continue;
            if (hipMalloc(&g.dev, g.image.size()) != hipSuccess) {
                g.dev = nullptr;
                return set_error(TVS_E_NOMEM, "hipMalloc of the batch work list failed");
            }
            g.owned = true;
            TVS_HIP_TRY(hipMemcpy(g.dev, g.image.data(), g.image.size(), hipMemcpyHostToDevice));
        }
        return TVS_OK;
    }
    size_t total = 0;
    std::vector<size_t> off;
    for (auto& g : bp->groups) {
        off.push_back(total);
        total += (g.image.size() + 255) & ~(size_t)255;
    }
    if (total == 0) return TVS_OK;
    if (ext->capacity < total) {
        size_t cap = std::max(total, 2 * ext->capacity);
        if (ext->dev) (void)hipFree(ext->dev);
        if (ext->host) (void)hipHostFree(ext->host);
        ext->dev = ext->host = nullptr;
        ext->capacity = 0;
        if (hipMalloc(&ext->dev, cap) != hipSuccess) {
            ext->dev = nullptr;
            return set_error(TVS_E_NOMEM, "hipMalloc of the batch work lists failed");
        }
        if (hipHostMalloc(&ext->host, cap, hipHostMallocDefault) != hipSuccess) {
            ext->host = nullptr;
            return set_error(TVS_E_NOMEM, "hipHostMalloc of the batch staging failed");
        }
        ext->capacity = cap;
    }
    for (size_t i = 0; i < bp->groups.size(); ++i) {
        auto& g = bp->groups[i];
        if (g.image.empty()) continue;
        std::memcpy((char*)ext->host + off[i], g.image.data(), g.image.size());
        g.dev = (char*)ext->dev + off[i];
        g.owned = false;
    }
    TVS_HIP_TRY(hipMemcpyAsync(ext->dev, ext->host, total, hipMemcpyHostToDevice, st));
    return TVS_OK;
}

// Host work and uploads for the whole batch (no stream work).
int prepare_batch(int n, tvs_plan* const* plans, void* const* grids, const double* const* coeffs,
                  const int64_t* T, BatchPlan* bp) {
    std::map<Variant, std::vector<Member>> groups;
    for (int i = 0; i < n; ++i) {
        tvs_plan* p = plans[i];
        if (T[i] == 0) continue;
        int rc = ensure_scratch(p);
        if (rc) return rc;
        if (p->prob.dependence == TVS_GAUSS_SEIDEL) {
            bp->gs.emplace_back(p, i);
            continue;
        }
        const Schedule s = member_schedule(p->prob, p->sched, T[i]);
        // equal weights take the shared-product tile body in round launches
        const int uni = !persistent_mode() && same_weight_bits(coeffs[i], p->prob.order) ? 1 : 0;
        Variant v{p->prob.dtype, p->prob.ndim, p->prob.shape, p->prob.boundary, uni,
                  p->prob.ndim == 1 ? 0 : s.c};
        groups[v].push_back(Member{p, grids[i], coeffs[i], T[i], s});
    }
    set_lds_attributes<double>();
    set_lds_attributes<float>();
    for (auto& kv : groups) {
        GroupLaunch gl;
        int rc = kv.first.dtype == TVS_F64 ? prepare_group<double>(kv.first, kv.second, &gl)
                                           : prepare_group<float>(kv.first, kv.second, &gl);
        bp->groups.push_back(gl);
        if (rc) return rc;
    }
    return TVS_OK;
}

// Enqueue a prepared batch on st: the Jacobi groups, and (with_gs) the
// Gauss-Seidel members, which run through their own persistent kernel and
// are kept out of captured graphs.  With ext->naux > 0 the Gauss-Seidel
// members are spread over ext's auxiliary streams, after everything already
// on st, and st waits for all of them.
int launch_batch(const BatchPlan& bp, void* const* grids, const double* const* coeffs,
                 const int64_t* T, hipStream_t st, bool with_gs, const BatchBuffers* ext = nullptr) {
    for (const auto& g : bp.groups) {
        int rc = g.v.dtype == TVS_F64 ? launch_group<double>(g, st) : launch_group<float>(g, st);
        if (rc) return rc;
    }
    if (!with_gs || bp.gs.empty()) return TVS_OK;
    const int naux = ext ? std::min<int>(ext->naux, (int)bp.gs.size()) : 0;
    if (naux > 1) {
        TVS_HIP_TRY(hipEventRecord(ext->fork, st));
        for (int a = 0; a < naux; ++a) TVS_HIP_TRY(hipStreamWaitEvent(ext->aux[a], ext->fork, 0));
    }
    for (size_t i = 0; i < bp.gs.size(); ++i) {
        const auto& m = bp.gs[i];
        CoeffBuf cb;
        fill_coeffs(m.first->prob, coeffs[m.second], &cb);
        hipStream_t s = naux > 1 ? ext->aux[i % naux] : st;
        int rc = enqueue_gs(m.first, grids[m.second], cb, T[m.second], s);
        if (rc) return rc;
    }
    if (naux > 1)
        for (int a = 0; a < naux; ++a) {
            TVS_HIP_TRY(hipEventRecord(ext->join[a], ext->aux[a]));
            TVS_HIP_TRY(hipStreamWaitEvent(st, ext->join[a], 0));
        }
    return TVS_OK;
}

// ---------------------------------------------------------------------------
// graph cache: a batch layout that repeats (same plans, grids, step counts
// and weights) is captured once and replayed
// ---------------------------------------------------------------------------
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    BatchPlan bp;
    std::vector<tvs_plan*> plans;
};
constexpr size_t kMaxGraphs = 32;

std::mutex g_graph_mu;
std::map<std::vector<double>, GraphEntry> g_graphs;

// Side streams on which a batch runs its Gauss-Seidel members next to the
// captured Jacobi rounds and next to each other (each member is one chain of
// dependent columns that fills little of the chip).  One set per device, kept
// until the process ends; used under g_graph_mu.
struct GsSide {
    static constexpr int kAux = 4;
    hipStream_t aux[kAux] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kAux] = {};
};
std::map<int, GsSide> g_gs_side;

GsSide* gs_side(int dev) {
    auto it = g_gs_side.find(dev);
    if (it != g_gs_side.end()) return &it->second;
    GsSide side;
    bool ok = hipEventCreateWithFlags(&side.fork, hipEventDisableTiming) == hipSuccess;
    for (int a = 0; ok && a < GsSide::kAux; ++a)
        ok = hipStreamCreateWithFlags(&side.aux[a], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&side.join[a], hipEventDisableTiming) == hipSuccess;
    if (!ok) return nullptr;  // members then run on the batch stream
    return &g_gs_side.emplace(dev, side).first->second;
}

std::vector<double> layout_key(int n, tvs_plan* const* plans, void* const* grids,
                               const double* const* coeffs, const int64_t* T, int device) {
    std::vector<double> key;
    key.push_back(device);
    key.push_back(persistent_mode() ? 1 : 0);
    for (int i = 0; i < n; ++i) {
        key.push_back((double)(uintptr_t)plans[i]);
        key.push_back((double)(uintptr_t)grids[i]);
        key.push_back((double)T[i]);
        for (int q = 0; q < plans[i]->prob.order; ++q) key.push_back(coeffs[i][q]);
    }
    return key;
}

}  // namespace

void graph_cache_drop(tvs_plan* p) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
        bool uses = std::find(it->second.plans.begin(), it->second.plans.end(), p) !=
                    it->second.plans.end();
        if (uses) {
            (void)hipGraphExecDestroy(it->second.exec);
            free_batch(&it->second.bp);
            it = g_graphs.erase(it);
        } else {
            ++it;
        }
    }
}

int batch_run(int n, tvs_plan* const* plans, void* const* grids, const double* const* coeffs,
              const int64_t* T, hipStream_t st, bool use_graph, BatchBuffers* ext) {
    if (ext) {  // asynchronous: work lists in the caller's buffers, nothing waited for
        BatchPlan bp;
        int rc = prepare_batch(n, plans, grids, coeffs, T, &bp);
        if (rc == TVS_OK) rc = upload_batch(&bp, ext, st);
        if (rc == TVS_OK) rc = launch_batch(bp, grids, coeffs, T, st, true, ext);
        return rc;
    }
    if (!use_graph) {
        BatchPlan bp;
        int rc = prepare_batch(n, plans, grids, coeffs, T, &bp);
        if (rc == TVS_OK) rc = upload_batch(&bp, nullptr, st);
        if (rc == TVS_OK) rc = launch_batch(bp, grids, coeffs, T, st, true);
        // the work lists must outlive the launches that read them
        if (hipStreamSynchronize(st) != hipSuccess && rc == TVS_OK)
            rc = set_error(TVS_E_DEVICE, "batch launch failed");
        if (int* bs = batch_status_host();
            rc == TVS_OK && bs && __atomic_exchange_n(bs, 0, __ATOMIC_ACQ_REL) != 0)
            rc = set_error(TVS_E_DEVICE, "a batch launch timed out waiting for a band");
        free_batch(&bp);
        return rc;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto key = layout_key(n, plans, grids, coeffs, T, dev);
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        if (g_graphs.size() >= kMaxGraphs) {  // drop one cached layout
            auto victim = g_graphs.begin();
            (void)hipStreamSynchronize(st);
            (void)hipGraphExecDestroy(victim->second.exec);
            free_batch(&victim->second.bp);
            g_graphs.erase(victim);
        }
        GraphEntry e;
        int rc = prepare_batch(n, plans, grids, coeffs, T, &e.bp);
        if (rc == TVS_OK) rc = upload_batch(&e.bp, nullptr, st);
        if (rc) {
            free_batch(&e.bp);
            return rc;
        }
        hipStream_t cap;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
            free_batch(&e.bp);
            return set_error(TVS_E_DEVICE, "stream creation failed");
        }
        hipGraph_t graph = nullptr;
        hipError_t eb = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (eb == hipSuccess) rc = launch_batch(e.bp, grids, coeffs, T, cap, false);
        hipError_t ec = eb == hipSuccess ? hipStreamEndCapture(cap, &graph) : eb;
        (void)hipStreamDestroy(cap);
        if (rc || ec != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            free_batch(&e.bp);
            return rc ? rc : set_error(TVS_E_DEVICE, "batch graph capture failed");
        }
        ec = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ec != hipSuccess) {
            free_batch(&e.bp);
            return set_error(TVS_E_DEVICE, "batch graph instantiation failed");
        }
        e.plans.assign(plans, plans + n);
        it = g_graphs.emplace(std::move(key), std::move(e)).first;
    }
    // Gauss-Seidel members run eagerly (outside the graph) on side streams
    // forked from the batch stream, concurrently with the Jacobi rounds, and
    // are joined back before the batch stream continues
    const auto& gs = it->second.bp.gs;
    GsSide* side = gs.empty() ? nullptr : gs_side(dev);
    if (side) {
        TVS_HIP_TRY(hipEventRecord(side->fork, st));
        for (int a = 0; a < GsSide::kAux; ++a)
            TVS_HIP_TRY(hipStreamWaitEvent(side->aux[a], side->fork, 0));
    }
    int rc = TVS_OK;
    for (size_t i = 0; i < gs.size() && rc == TVS_OK; ++i) {
        const auto& m = gs[i];
        CoeffBuf cb;
        fill_coeffs(m.first->prob, coeffs[m.second], &cb);
        rc = enqueue_gs(m.first, grids[m.second], cb, T[m.second],
                        side ? side->aux[i % GsSide::kAux] : st);
    }
    TVS_HIP_TRY(hipGraphLaunch(it->second.exec, st));
    if (side)
        for (int a = 0; a < GsSide::kAux; ++a) {
            TVS_HIP_TRY(hipEventRecord(side->join[a], side->aux[a]));
            TVS_HIP_TRY(hipStreamWaitEvent(st, side->join[a], 0));
        }
    return rc;
}

}  // namespace tvs

using namespace tvs;

extern "C" int stencil_batch_run(int n, tvs_plan* const* plans, void* const* grids,
                                 const double* const* coeffs, const int64_t* T, void* stream) {
    clear_error();
    if (n < 0) return set_error(TVS_E_INVALID, "n < 0");
    if (n == 0) return TVS_OK;
    if (!plans || !grids || !coeffs || !T) return set_error(TVS_E_INVALID, "NULL argument");
    if (n > 60000) return set_error(TVS_E_INVALID, "batch larger than 60000 grids");
    for (int i = 0; i < n; ++i) {
        if (plans[i] && plans[i]->prob.rule == TVS_RULE_LIFE)
            return set_error(TVS_E_UNSUPPORTED, "Game of Life plans do not run in batches");
        if (plans[i] && plans[i]->prob.radius > 1)
            return set_error(TVS_E_UNSUPPORTED, "plans of radius > 1 do not run in batches");
        if (!plans[i] || !grids[i] || !coeffs[i]) return set_error(TVS_E_INVALID, "NULL member");
        if (T[i] < 0) return set_error(TVS_E_INVALID, "T < 0");
    }
    // a plan or grid given twice would share scratch and data between members
    // that run at the same time
    {
        std::vector<const void*> seen;
        for (int i = 0; i < n; ++i)
            if (T[i] > 0) {
                seen.push_back(plans[i]);
                seen.push_back(grids[i]);
            }
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
            return set_error(TVS_E_INVALID, "a plan or grid appears twice in the batch");
    }
    for (int i = 0; i < n; ++i)
        if (plans[i]->prob.dependence == TVS_GAUSS_SEIDEL && T[i] > 0) {
            int rc = gs_report_previous(plans[i]);
            if (rc) return rc;
        }
    // a persistent batch launch whose bounded wait expired (reported once)
    if (int* bs = batch_status_host(); bs && __atomic_exchange_n(bs, 0, __ATOMIC_ACQ_REL) != 0)
        return set_error(TVS_E_DEVICE, "an earlier batch launch timed out waiting for a band; "
                                       "its results are invalid");
    const char* env = std::getenv("TVS_BATCH_GRAPH");
    const bool use_graph = !(env && env[0] == '0');
    int rc = batch_run(n, plans, grids, coeffs, T, (hipStream_t)stream, use_graph, nullptr);
    if (rc) return rc;
    for (int i = 0; i < n; ++i)
        if (plans[i]->prob.dependence == TVS_GAUSS_SEIDEL && T[i] > 0) {
            rc = gs_queue_status_copy(plans[i], (hipStream_t)stream);
            if (rc) return rc;
        }
    return TVS_OK;
}
