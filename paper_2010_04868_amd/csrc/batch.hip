// Batched launches: many Jacobi grids of uneven shapes and step counts
// advance together.
//
// A batch is cut into band rounds: round b runs band b of every grid that
// still has one, as ONE kernel launch whose workgroups take (grid, tile)
// items from a device-resident work list.  The kernel boundary between
// rounds is the only synchronization a band needs (band b+1 reads what band
// b wrote and overwrites what band b read), so there are no waits between
// workgroups and nothing to deadlock.  The round sequence of a batch layout
// that repeats is captured once in a hipGraph and replayed.
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

constexpr int kBatchC = 4;    // nD: points per lane
constexpr int kBatchNPT = 4;  // nD: staging values per thread (any k >= 1)

struct BatchItem {
    unsigned int g;
    unsigned int b;
    unsigned int t;
    unsigned int pad;
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

template <typename T, int D, bool BOX, bool PER, bool UNI>
__global__ __launch_bounds__(512) void batch_round_nd(const GridNd<T>* grids,
                                                      const BatchItem* items, int round) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const BatchItem w = items[blockIdx.x];
    const GridNd<T>& gr = grids[w.g];
    const int which = round == gr.nbands - 1 ? 1 : 0;
    nd::tstp_tile<T, D, BOX, PER, kBatchC, kBatchNPT, UNI>(
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
    int dtype, ndim, shape, boundary, uniform;
    bool operator<(const Variant& o) const {
        return std::tie(dtype, ndim, shape, boundary, uniform) <
               std::tie(o.dtype, o.ndim, o.shape, o.boundary, o.uniform);
    }
};

struct Member {
    tvs_plan* plan;
    void* grid;
    const double* coeffs;
    int64_t T;
};

// Schedule the batch uses for a grid: fixed lane width, depth min(k, T).
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
        Schedule s = batch_schedule(p);
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
    // round b: band b of every grid that has one; items of a round are contiguous
    int maxb = 0;
    for (int v : nb) maxb = std::max(maxb, v);
    for (int b = 0; b < maxb; ++b) {
        round_begin->push_back((int)items->size());
        for (size_t i = 0; i < ms.size(); ++i)
            if (b < nb[i])
                for (int t = 0; t < tiles_per_band[i][b]; ++t)
                    items->push_back(BatchItem{(unsigned)i, (unsigned)b, (unsigned)t, 0u});
    }
    round_begin->push_back((int)items->size());
    *lds_out = lds;
    return TVS_OK;
}

// One group, prepared on the host.  Its work list ([items | grids]) is
// built as a host image and then uploaded either into memory the group owns
// (synchronously, before any stream work, so that the launches can be
// captured in a graph) or into caller-provided buffers (asynchronously).
struct GroupLaunch {
    Variant v;
    void* dev = nullptr;  // [items | grids]
    bool owned = false;   // dev was allocated for this group
    std::vector<unsigned char> image;
    size_t lds = 0;
    std::vector<int> round_begin;  // item offset of each round, plus the end
    size_t off_grids = 0;
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
    gl->off_grids = (items.size() * sizeof(BatchItem) + 255) & ~(size_t)255;
    const size_t grid_bytes =
        v.ndim == 1 ? g1d.size() * sizeof(Grid1d<T>) : gnd.size() * sizeof(GridNd<T>);
    const size_t total = gl->off_grids + grid_bytes;
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

template <typename T>
int launch_group(const GroupLaunch& gl, hipStream_t st) {
    if (!gl.dev || gl.image.empty()) return TVS_OK;
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
#define TVS_B(DD, B, PR, U) go(batch_round_nd<T, DD, B, PR, U>)
#define TVS_B3(DD)                                                                              \
    if (box) {                                                                                  \
        if (per) { if (uni) TVS_B(DD, true, true, true); else TVS_B(DD, true, true, false); }   \
        else { if (uni) TVS_B(DD, true, false, true); else TVS_B(DD, true, false, false); }     \
    } else {                                                                                    \
        if (per) { if (uni) TVS_B(DD, false, true, true); else TVS_B(DD, false, true, false); } \
        else { if (uni) TVS_B(DD, false, false, true); else TVS_B(DD, false, false, false); }   \
    }
            if (v.ndim == 2) { TVS_B3(2) } else { TVS_B3(3) }
#undef TVS_B3
#undef TVS_B
        }
        TVS_HIP_TRY(hipGetLastError());
    }
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
    static bool done = false;
    if (done) return;
    done = true;
    auto set = [](auto kern) {
        (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
    };
    set(batch_round_nd<T, 2, true, true, true>);   set(batch_round_nd<T, 2, true, true, false>);
    set(batch_round_nd<T, 2, true, false, true>);  set(batch_round_nd<T, 2, true, false, false>);
    set(batch_round_nd<T, 2, false, true, true>);  set(batch_round_nd<T, 2, false, true, false>);
    set(batch_round_nd<T, 2, false, false, true>); set(batch_round_nd<T, 2, false, false, false>);
    set(batch_round_nd<T, 3, true, true, true>);   set(batch_round_nd<T, 3, true, true, false>);
    set(batch_round_nd<T, 3, true, false, true>);  set(batch_round_nd<T, 3, true, false, false>);
    set(batch_round_nd<T, 3, false, true, true>);  set(batch_round_nd<T, 3, false, true, false>);
    set(batch_round_nd<T, 3, false, false, true>); set(batch_round_nd<T, 3, false, false, false>);
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
        Variant v{p->prob.dtype, p->prob.ndim, p->prob.shape, p->prob.boundary,
                  same_weight_bits(coeffs[i], p->prob.order) ? 1 : 0};
        groups[v].push_back(Member{p, grids[i], coeffs[i], T[i]});
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

// Enqueue a prepared batch on st: the Jacobi rounds, and (with_gs) the
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
