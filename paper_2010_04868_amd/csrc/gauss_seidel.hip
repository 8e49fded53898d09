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
//     a running wave (no deadlock for any grid size); progress (steps
//     completed) is published to the items that depend on it, and band data
//     crosses the XCDs' separate L2 caches through agent-scope loads and
//     stores, so that no fence has to invalidate or write back an L2;
//   * every wait is bounded; on expiry the kernel records a status word and
//     the remaining waits return at once, so the launch always drains.
// Band layout: a run first copies the interior rows into a layout of its
// own and copies them back at the end.  Band b holds its 64 rows column by
// column, and row r is shifted right by SIG*r columns: element (x0+r, y) sits
// at lay[((b*Wp) + y + SIG*r)*64 + r], Wp = n1 + 63*SIG.  The 64 points that
// a wave updates in one step (row r at column c+1 = u - SIG*r) then share one
// layout column and occupy 64 consecutive elements, so every load and store
// of a step is one contiguous 512-byte (FP64) access instead of 64 accesses
// to 64 rows.  The top border row is read from the grid itself; the bottom
// one is copied once into an extra band slot (row 0 of band nb), so that the
// row below any band is in the layout with the same column stride.
// Each point is updated exactly once per sweep, with the canonical operation
// order, after all of its "new" and before any of its "old" neighbours are
// overwritten, so the result is bit-identical to the naive lexicographic
// sweep.
#include "gs_order.hpp"
#include "kernels.hpp"

namespace tvs {
namespace {

constexpr int kRows = 64;        // rows per band (one wave)
constexpr int kBlock = 8;        // steps whose loads are issued together
// Steps between dependency checks and progress updates (KS, a template
// parameter chosen by row width).  A dependent item trails its producer by
// about KS columns, so short intervals keep more items in flight; each check
// costs a progress load and each update a wait for the item's stores.  Rows
// of 2048 columns or more take 16, narrower ones 8 (measured on 600^2 to
// 4096^2 grids once the polls no longer contend, see gs_reset).
constexpr long long kSpinLimit = 1ll << 22;  // ~seconds: far beyond any legitimate wait
constexpr int kAllSteps = 1 << 30;            // progress of a finished item

struct GsArgs {
    int n0, n1;
    int nb;       // bands of interior rows
    int sweeps;   // sweeps in this launch
    int ncols;    // interior columns
    int nitems;
    int Wp;       // layout columns per band row
    int* ticket;
    int* status;
    int* progress;  // [sweeps][nb], one counter per kProgStride ints
};

__device__ __forceinline__ int load_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Band data that other items read or wrote moves with agent-scope (sc1)
// loads and stores: each is coherent across the XCDs' L2 caches by itself
// (the same accesses a relaxed agent-scope atomic makes), so an item's waits
// need no acquire fence (an L2 invalidate) and its progress stores no
// release fence (an L2 write-back).  What remains of release is that the
// item's own stores have completed before the progress store that announces
// them (vmcnt(0)); of acquire, that its loads are issued after the progress
// loads have returned.  The compiler barriers keep the accesses on their side.
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The value `lane` holds (the same in every lane).
template <typename T>
__device__ __forceinline__ T read_lane(T v, int lane) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
    }
}
// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maximum), gfx9 encoding
constexpr int kWaitVmcnt0 = 0x0F70;
__device__ __forceinline__ void after_waits() { asm volatile("" ::: "memory"); }
__device__ __forceinline__ void before_progress_store() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    asm volatile("" ::: "memory");
}

// Wait until *p >= need (or the launch has been aborted).  Uniform per wave.
// Relaxed polling: the caller issues one acquire fence after all its waits.
// The status word, one line read by every waiting wave of the launch, is
// read every 64 polls only.
__device__ __forceinline__ void wait_at_least(const int* p, int need, int* status) {
    long long spins = 0;
    while (load_relaxed(p) < need) {
        if ((spins & 63) == 63 &&
            __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            return;
        if (++spins > kSpinLimit) {
            __hip_atomic_store(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// The 2D kernel's progress counters sit one per cache line: the waves that
// poll a counter and the item that publishes it then share that line with
// no other counter's traffic (packed 32 to a line, their agent-scope polls
// and stores all queued on the same lines).
constexpr int kProgStride = 32;  // ints: 128 bytes

__global__ void gs_reset(int* ticket, int* progress, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *ticket = 0;
    for (; i < n; i += gridDim.x * blockDim.x) progress[(int64_t)i * kProgStride] = 0;
}

// Column y of the row above / below the band, in whichever array holds it.
template <typename T>
struct GsRows {
    const T* north;  // row x0-1: band b-1's last row in the layout, or grid row 0
    int64_t nstride; // element step per column of `north`
    const T* south;  // row x0+rows: band b+1's first row in the layout, or grid row n0-1
    int64_t sstride;
};

template <typename T, bool BOX, int KS>
__global__ __launch_bounds__(64) void gs2d(T* grid, T* lay, GsArgs a, Coeffs<T> cf) {
    constexpr int SIG = BOX ? 2 : 1;
    static_assert(KS % kBlock == 0 && kBlock % 2 == 0, "sync interval; even block starts");
    const int lane = threadIdx.x;
    const int n1 = a.n1;
    const int64_t Wp = a.Wp;
    for (;;) {
        // No branch on the lane index may sit in this loop: given a region
        // that only lane 0 enters, the compiler may send lanes 1..63 round a
        // shorter back edge that skips it, and they would then re-read a stale
        // ticket without lane 0 and repeat an item forever.  So every lane
        // joins the ticket atomic (lane 0 adds 1, the others 0) and the
        // progress stores, and the ticket is made a scalar.
        const int mine = atomicAdd(a.ticket, lane == 0 ? 1 : 0);
        const int item = __builtin_amdgcn_readfirstlane(mine);
        if (item >= a.nitems) break;
        int b, t;
        gs::decode_item(item, a.nb, a.sweeps, &b, &t);
        const int x0 = 1 + kRows * b;
        const int rows = min(kRows, a.n0 - 1 - x0);
        const int L = rows - 1;  // last row of the band
        const bool active = lane < rows;
        T* band = lay + (int64_t)b * Wp * kRows;
        // neighbour rows of the band; column y of north is north[y * nstride]
        GsRows<T> nb_;
        if (b > 0) {
            nb_.north = lay + ((int64_t)(b - 1) * Wp + SIG * (kRows - 1)) * kRows + (kRows - 1);
            nb_.nstride = kRows;
        } else {
            nb_.north = grid;
            nb_.nstride = 1;
        }
        // band b+1's first row, or the bottom border row in band slot nb
        nb_.south = lay + (int64_t)(b + 1) * Wp * kRows;
        nb_.sstride = kRows;
        // column y of this lane's row and of the row below it
        auto own = [&](int y) -> T* { return band + (int64_t)(y + SIG * lane) * kRows + lane; };
        auto below = [&](int y) -> const T* {
            return lane < L ? band + (int64_t)(y + SIG * (lane + 1)) * kRows + lane + 1
                            : nb_.south + (int64_t)y * nb_.sstride;
        };
        auto above = [&](int y) -> const T* {
            return lane > 0 ? band + (int64_t)(y + SIG * (lane - 1)) * kRows + lane - 1
                            : nb_.north + (int64_t)y * nb_.nstride;
        };
        // registers: west (new), centre/east (old), north and south histories;
        // seh: the south-east values of the last SIG steps (step u in slot
        // u mod SIG: intervals and blocks start at even steps)
        T Wv = 0, Cv = 0, out = 0;
        T seh[SIG];
#pragma unroll
        for (int i = 0; i < SIG; ++i) seh[i] = T(0);
        T Ev = active ? ld_agent(own(0)) : T(0);
        T NWv, Nv, NEv, SWv, Sv, SEv;
        NWv = Nv = NEv = active ? ld_agent(above(0)) : T(0);
        SWv = Sv = SEv = active ? ld_agent(below(0)) : T(0);
        auto counter = [&](int tt, int bb) { return a.progress + (int64_t)(tt * a.nb + bb) * kProgStride; };
        int* prog_self = counter(t, b);
        const int* prog_north = b > 0 ? counter(t, b - 1) : nullptr;
        const int* prog_prev = t > 0 ? counter(t - 1, b) : nullptr;
        const int* prog_south = (t > 0 && b + 1 < a.nb) ? counter(t - 1, b + 1) : nullptr;

        // steps: at step u, lane i updates column u - SIG*i (c = u - 1 - SIG*i
        // in [-1, ncols]).  Progress is published as the number of steps an
        // item has completed (kAllSteps once it is done).  Before an interval
        // of steps [us, us+KS) an item waits, per producer, for exactly the
        // steps whose values the interval reads:
        //  * (b, t-1), the same band one sweep earlier: lane i reads the old
        //    value of its own row at column u - SIG*i + 1 (written by that
        //    item's lane i at its step u + 1) and of row i+1 (its lane i+1,
        //    step u + 1 + SIG): at most us + KS + SIG + 1 steps;
        //  * (b+1, t-1), the band below one sweep earlier: only the last lane
        //    reads its first row, at column u - SIG*L + 1 (that item's lane 0,
        //    step u - SIG*L + 1): us + KS + 1 - SIG*L steps, which is behind
        //    this item's own position;
        //  * (b-1, t), the band above in this sweep: lane 0 reads its last row
        //    (lane 63) at column u - 1 + SIG, written at that item's step
        //    u - 1 + SIG + 63*SIG: us + KS - 1 + 64*SIG steps.
        // These also keep every overwrite behind the reads of the old values
        // it replaces: (b-1, t) reads this band's first row, and (b+1, t-1)
        // its last row, before this item overwrites them.
        const int U = a.ncols + 2 + SIG * L;
        for (int us = 0; us < U; us += KS) {
          if (prog_prev) wait_at_least(prog_prev, us + KS + SIG + 1, a.status);
          if (prog_south && us + KS + 1 - SIG * L > 0)
              wait_at_least(prog_south, us + KS + 1 - SIG * L, a.status);
          if (prog_north) wait_at_least(prog_north, us + KS - 1 + SIG * kRows, a.status);
          // the producers' rows written before their progress stores are visible now
          after_waits();
          // An inner interval keeps every lane (idle ones included) on an
          // interior column, 0 <= c < ncols, for all of its steps: it needs no
          // test per step, and idle lanes of a partial band store into their
          // own unused row slots.
          const bool inner = us >= 1 + SIG * (kRows - 1) && us + KS <= a.ncols + 1;
          auto interval = [&](auto inner_t) {
            constexpr bool IN = decltype(inner_t)::value;
            // The loads of a block of kBlock steps: east and south values of
            // every lane's point and lane 0's north values.  They read only
            // values the waits above cover, and old values no lane overwrites
            // before the block's steps, so they may be issued a block early.
            auto load_blk = [&](int u0, T (&e_in)[kBlock], T (&se_in)[kBlock], T (&n_in)[kBlock]) {
#pragma unroll
              for (int m = 0; m < kBlock; ++m) {
                  const int c = u0 + m - 1 - SIG * lane;
                  const int ye = c + 2;
                  const int yn = c + SIG;
                  const bool ok = active && c >= -1 && ye <= n1 - 1;
                  // invalid lanes read a harmless in-band element and drop it
                  const T e = ld_agent(ok ? own(ye) : band);
                  const T se = ld_agent(ok ? below(ye) : band);
                  e_in[m] = ok ? e : T(0);
                  se_in[m] = ok ? se : T(0);
                  const bool okn = lane == 0 && c >= -1 && yn <= n1 - 1;
                  const T nv = ld_agent(okn ? above(yn) : band);
                  n_in[m] = okn ? nv : T(0);
              }
            };
            // Step u: nin is the value of the row above one column ahead of
            // where it was last step (lane i-1's last output; for lane 0 the
            // north row), ein the east value, sein the south-east one.
            auto step = [&](int u, T nin, T ein, T sein, auto inner_s) {
                  constexpr bool IS = decltype(inner_s)::value;
                  const int c = u - 1 - SIG * lane;
                  if (IS || (c >= -1 && c <= a.ncols)) {
                      if (BOX) {
                          NWv = Nv;
                          Nv = NEv;
                          NEv = nin;
                          SWv = Sv;
                          Sv = SEv;
                          SEv = sein;
                      } else {
                          Nv = nin;
                          Sv = SEv;
                          SEv = sein;
                      }
                      Cv = Ev;
                      Ev = ein;
                      T r = Cv;  // border columns pass their fixed value along
                      if (IS || (c >= 0 && c < a.ncols)) {
                          if (BOX) {
                              r = cf.c[0] * NWv;
                              r = r + cf.c[1] * Nv;
                              r = r + cf.c[2] * NEv;
                              r = r + cf.c[3] * Wv;
                              r = r + cf.c[4] * Cv;
                              r = r + cf.c[5] * Ev;
                              r = r + cf.c[6] * SWv;
                              r = r + cf.c[7] * Sv;
                              r = r + cf.c[8] * SEv;
                          } else {
                              r = cf.c[0] * Nv;
                              r = r + cf.c[1] * Wv;
                              r = r + cf.c[2] * Cv;
                              r = r + cf.c[3] * Ev;
                              r = r + cf.c[4] * Sv;
                          }
                          if (IS || active) st_agent(own(c + 1), r);
                      }
                      Wv = r;
                      out = r;
                  }
            };
            // Steps of a block outside inner intervals: every lane loads its
            // own east value.  seh keeps the south-east values of the last
            // SIG steps for the inner interval that may follow.
            auto comp_blk = [&](int u0, const T (&e_in)[kBlock], const T (&se_in)[kBlock],
                                const T (&n_in)[kBlock]) {
#pragma unroll
              for (int m = 0; m < kBlock; ++m) {
                  const T nin = shift_up<64>(out, n_in[m]);
                  seh[m % SIG] = se_in[m];
                  step(u0 + m, nin, e_in[m], se_in[m], std::false_type{});
              }
            };
            if constexpr (IN) {
              // An inner interval issues every load of its KS steps at once,
              // right after its waits: the south-east values of each step,
              // and lane 0's east and north values with one load each
              // (lane j holds step us + j's), read back with readlane.
              // (lane 0's values first: the counter of outstanding loads
              // drains in issue order)
              T e_vec = T(0), n_vec = T(0);
              if (lane < KS) {
                  e_vec = ld_agent(band + (int64_t)(us + 1 + lane) * kRows);
                  n_vec = ld_agent(nb_.north + (int64_t)(us - 1 + SIG + lane) * nb_.nstride);
              }
              // the row below at column us+1-SIG*lane onwards (lane L: the
              // south row); column strides are whole layout columns
              T se_all[KS];
              const T* bptr = lane < L ? band + (int64_t)(us + 1 + SIG) * kRows + lane + 1
                                       : nb_.south + (int64_t)(us + 1 - SIG * lane) * kRows;
#pragma unroll
              for (int m = 0; m < KS; ++m) se_all[m] = ld_agent(bptr + m * kRows);
#pragma unroll
              for (int m = 0; m < KS; ++m) {
                  const T n0 = read_lane(n_vec, m), e0 = read_lane(e_vec, m);
                  const T nin = shift_up<64>(out, n0);
                  const T ein = shift_up<64>(seh[m % SIG], e0);
                  seh[m % SIG] = se_all[m];
                  step(us + m, nin, ein, se_all[m], std::true_type{});
              }
              return;
            }
            // blocks of the interval (the last interval stops at U), the next
            // block's loads in flight while a block computes
            const int uend = min(us + KS, U);
            T eA[kBlock], seA[kBlock], nA[kBlock], eB[kBlock], seB[kBlock], nB[kBlock];
            load_blk(us, eA, seA, nA);
            for (int u0 = us; u0 < uend; u0 += 2 * kBlock) {
              const bool hasB = u0 + kBlock < uend;
              if (hasB) load_blk(u0 + kBlock, eB, seB, nB);
              comp_blk(u0, eA, seA, nA);
              if (!hasB) break;
              if (u0 + 2 * kBlock < uend) load_blk(u0 + 2 * kBlock, eA, seA, nA);
              comp_blk(u0 + kBlock, eB, seB, nB);
            }
          };
          if (inner)
              interval(std::true_type{});
          else
              interval(std::false_type{});
          // publish the steps completed
          before_progress_store();
          __hip_atomic_store(prog_self, us + KS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        before_progress_store();
        __hip_atomic_store(prog_self, kAllSteps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Grid <-> band layout, one 64 x 64 tile of (layout column, row) per
// workgroup.  Row r of the tile covers grid columns starting at J - SIG*r,
// so both the grid rows and the layout columns are accessed contiguously;
// the tile passes through LDS (row stride 65 against bank conflicts).
template <typename T, int SIG, bool IN>
__global__ __launch_bounds__(256) void gs_layout(T* grid, T* lay, int n0, int n1, int64_t Wp,
                                                 int ntiles) {
    __shared__ T tile[kRows][kRows + 1];
    const int b = blockIdx.x / ntiles;
    const int J = (blockIdx.x % ntiles) * kRows;  // first layout column of the tile
    const int x0 = 1 + kRows * b;
    const int rows = min(kRows, n0 - 1 - x0);
    const int tid = threadIdx.x;
    T* band = lay + (int64_t)b * Wp * kRows;
    if (IN) {
        // grid rows -> tile[r][jj] = grid(x0+r, J + jj - SIG*r)
        for (int e = tid; e < kRows * kRows; e += 256) {
            const int r = e / kRows, jj = e % kRows;
            const int y = J + jj - SIG * r;
            if (r < rows && y >= 0 && y < n1) tile[r][jj] = grid[(int64_t)(x0 + r) * n1 + y];
        }
        __syncthreads();
        // tile -> layout columns J + jj, rows contiguous
        for (int e = tid; e < kRows * kRows; e += 256) {
            const int jj = e / kRows, r = e % kRows;
            const int y = J + jj - SIG * r;
            if (r < rows && y >= 0 && y < n1 && J + jj < Wp)
                band[(int64_t)(J + jj) * kRows + r] = tile[r][jj];
        }
    } else {
        for (int e = tid; e < kRows * kRows; e += 256) {
            const int jj = e / kRows, r = e % kRows;
            const int y = J + jj - SIG * r;
            if (r < rows && y >= 0 && y < n1 && J + jj < Wp)
                tile[r][jj] = band[(int64_t)(J + jj) * kRows + r];
        }
        __syncthreads();
        // interior columns only: the border columns never change
        for (int e = tid; e < kRows * kRows; e += 256) {
            const int r = e / kRows, jj = e % kRows;
            const int y = J + jj - SIG * r;
            if (r < rows && y >= 1 && y < n1 - 1) grid[(int64_t)(x0 + r) * n1 + y] = tile[r][jj];
        }
    }
}

// The bottom border row (fixed) into band slot nb, row 0, without skew.
template <typename T>
__global__ __launch_bounds__(256) void gs_bottom_row(const T* grid, T* lay, int n0, int n1,
                                                     int nb, int64_t Wp) {
    const int y = blockIdx.x * 256 + threadIdx.x;
    if (y < n1) lay[((int64_t)nb * Wp + y) * kRows] = grid[(int64_t)(n0 - 1) * n1 + y];
}

// 1D Gauss-Seidel: lanes are successive sweeps.  This is the paper's way of
// vectorizing a Gauss-Seidel stencil (Section 3.4): a vector holds points of
// different time steps, skewed along the space axis, and each lane runs the
// sequential x-chain of its own sweep.  Global lane g = 64*w + j holds sweep
// t0+g and updates x = q + 1 - 2g at its step q.  It needs the new value of
// x-1 (its own last output) and the old values of x and x+1, which are lane
// g-1's outputs of steps q-2 and q-1 (Section 3.2's legality rule with
// s = 2); within a wave they arrive by DPP shifts.  Up to 16 waves: 1024
// sweeps in one launch, in place (writes trail reads by 2k positions).
// One wave per workgroup, so that every wave has a SIMD to itself and a
// step costs only its dependency chain.  Wave w's lane 0 takes its inputs, the outputs of wave w-1's lane
// 63, from a ring in device memory, a block of kG1Block steps at a time:
// wave w-1 stores a block's values with agent-scope stores (coherent across
// the XCDs' L2 caches) and publishes its count of finished blocks once they
// have completed; wave w waits for that count, loads the block with
// agent-scope loads (lane l holds the inputs of steps 64s + l) and hands
// them to lane 0 with readlane.  A producer also waits until its consumer
// has finished the block whose slots it is about to overwrite (the ring
// holds kG1Ring blocks).  Wave 0 reads the grid itself; the last sweep's
// wave writes the grid behind every read.  Every wait is bounded: on expiry
// the status word is set and the remaining waits return at once.
constexpr int kG1Block = 256;  // steps per block
constexpr int kG1Ring = 8;     // blocks per ring
constexpr int kG1MaxWaves = 16;

__global__ void gs1d_reset(int* prog, int w) {
    if ((int)threadIdx.x < w) prog[threadIdx.x] = 0;
}

template <typename T>
__device__ __forceinline__ T lane_of(T v, int l) {
    if constexpr (sizeof(T) == 8) {
        const long long x = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), l);
        const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
    }
}

template <typename T>
__global__ __launch_bounds__(64) void gs1d_mc(T* u, int n, int k, Coeffs<T> cf, T* ring,
                                              int* prog, int* status) {
    constexpr int BS = kG1Block, NS = BS / 64, RS = kG1Ring * BS;
    __shared__ T rbuf[BS];        // lane 63's outputs of a block (the next wave's inputs)
    __shared__ T obuf[BS];        // the last sweep's outputs of a block
    __shared__ T scrap[64 + BS];  // destinations of the lanes that hand nothing on
    const int lane = threadIdx.x;
    const int w = blockIdx.x;
    const int W = gridDim.x;
    const int wl = (k - 1) / 64, jl = (k - 1) % 64;  // the last sweep's lane
    const int g = 64 * w + lane;
    const T ul = u[0], ur = u[n - 1];
    const T c0 = cf.c[0], c1 = cf.c[1], c2 = cf.c[2];
    const int b_end = ((n - 3) + 2 * (k - 1)) / BS;  // last block of the last sweep
    const T* in_ring = ring + (size_t)w * RS;
    T* out_ring = ring + (size_t)(w + 1) * RS;
    T* rout = lane == 63 ? rbuf : scrap + lane;
    T* obase = (w == wl && lane == jl) ? obuf : scrap + lane;
    T p1 = ul, p2 = ul;  // this lane's outputs of the last two steps
    // input of step q: wave 0 the grid value at q + 3, wave w > 0 ring slot q
    auto input = [&](int q) -> T {
        if (w == 0) {
            const int p = q + 3;
            return p < n ? u[p] : T(0);
        }
        return ld_agent(in_ring + (q + RS) % RS);
    };
    for (int b = 0; b <= b_end; ++b) {
        if (w > 0) wait_at_least(prog + w - 1, b + 1, status);
        if (w + 1 < W && b - kG1Ring + 2 > 0) wait_at_least(prog + w + 1, b - kG1Ring + 2, status);
        after_waits();
        // R_j, the input of step BS*b - 2 + j: lane l holds R_{64s+l} in r[s]
        T r[NS];
#pragma unroll
        for (int s2 = 0; s2 < NS; ++s2) r[s2] = input(BS * b - 2 + 64 * s2 + lane);
        const T rlast = input(BS * b - 2 + BS);
        static_for<0, BS>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            // old values of x (lane g-1, step q-2) and x+1 (step q-1)
            const T rm = lane_of(r[m / 64], m % 64);
            const T rm1 = m + 1 < BS ? lane_of(r[(m + 1) / 64 % NS], (m + 1) % 64) : rlast;
            const T C = shift_up<64>(p2, rm);
            T E = shift_up<64>(p1, rm1);
            const int q = BS * b + m;
            const int x = q + 1 - 2 * g;
            E = x == n - 2 ? ur : E;  // the right end is fixed
            T f = c0 * p1;            // x-1: this sweep's new value
            f = f + c1 * C;
            f = f + c2 * E;
            // computed by every lane, then selected: no branch in the step
            asm volatile("" : "+v"(f));
            const bool valid = x >= 1 && x <= n - 2;
            p2 = p1;
            p1 = valid ? f : ul;
            rout[m] = p1;
            obase[m] = p1;
        });
        __syncthreads();
        if (w + 1 < W) {
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) {
                const int q = BS * b + 64 * s2 + lane;
                st_agent(out_ring + q % RS, rbuf[64 * s2 + lane]);
            }
        }
        if (w == wl) {
#pragma unroll
            for (int s2 = 0; s2 < NS; ++s2) {
                const int x = BS * b + 64 * s2 + lane + 1 - 2 * (k - 1);
                if (x >= 1 && x <= n - 2) u[x] = obuf[64 * s2 + lane];
            }
        }
        before_progress_store();
        __hip_atomic_store(prog + w, b + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

// Work area: ticket, status word, progress counters for up to kMaxSweeps
// sweeps per launch, then the band layout.
constexpr int kMaxSweeps = 256;

int bands_of(const Problem& p) { return (int)((p.dims[0] - 2 + kRows - 1) / kRows); }
int64_t layout_width(const Problem& p) {
    return p.dims[1] + (int64_t)(kRows - 1) * (p.shape == TVS_BOX ? 2 : 1);
}
size_t state_bytes(const Problem& p) {
    const size_t raw =
        (size_t)(64 + (size_t)bands_of(p) * kMaxSweeps * kProgStride + 64) * sizeof(int);
    return (raw + 255) / 256 * 256;
}

template <typename T>
hipError_t launch_gs_t(const Problem& p, T* grid, const Coeffs<T>& cf, int sweeps, void* work,
                       hipStream_t st) {
    if (sweeps < 1 || sweeps > kMaxSweeps) return hipErrorInvalidValue;
    GsArgs a{};
    a.n0 = (int)p.dims[0];
    a.n1 = (int)p.dims[1];
    a.ncols = a.n1 - 2;
    a.nb = bands_of(p);
    a.sweeps = sweeps;
    a.nitems = a.nb * sweeps;
    a.Wp = (int)layout_width(p);
    int* w = (int*)work;
    a.ticket = w;
    a.status = w + 1;
    a.progress = w + 64;  // keep counters on their own cache lines
    T* lay = (T*)((char*)work + state_bytes(p));
    const int nprog = a.nb * sweeps;
    hipLaunchKernelGGL(gs_reset, dim3((unsigned)std::min(1024, (nprog + 255) / 256 + 1)),
                       dim3(256), 0, st, a.ticket, a.progress, nprog);
    // as many persistent waves as the device holds at once (one per
    // workgroup), at most 16 per CU: more items in flight (measured on
    // 4096^2 FP64: 3072 waves 203.8 GStencil/s, 2048 194.8, 1024 166.2)
    auto go = [&](auto kern) {
        int per_cu = 0, dev = 0, cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, 64, 0) !=
                hipSuccess || per_cu < 1)
            per_cu = 8;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int waves = std::min(a.nitems, std::min(per_cu, 16) * std::max(1, cus));
        hipLaunchKernelGGL(kern, dim3(waves), dim3(64), 0, st, grid, lay, a, cf);
    };
    // sync interval by row width (measured on 600^2 to 4096^2 grids)
    const bool box = p.shape == TVS_BOX;
    if (a.ncols >= 2048)
        box ? go(gs2d<T, true, 16>) : go(gs2d<T, false, 16>);
    else
        box ? go(gs2d<T, true, 8>) : go(gs2d<T, false, 8>);
    return hipGetLastError();
}

template <typename T, bool IN>
hipError_t layout_t(const Problem& p, T* grid, void* work, hipStream_t st) {
    const int64_t Wp = layout_width(p);
    T* lay = (T*)((char*)work + state_bytes(p));
    const int ntiles = (int)((Wp + kRows - 1) / kRows);
    const int64_t nblk = (int64_t)ntiles * bands_of(p);
    if (nblk > INT32_MAX) return hipErrorInvalidValue;
    dim3 g((unsigned)nblk);
    if (p.shape == TVS_BOX)
        hipLaunchKernelGGL((gs_layout<T, 2, IN>), g, dim3(256), 0, st, grid, lay, (int)p.dims[0],
                           (int)p.dims[1], Wp, ntiles);
    else
        hipLaunchKernelGGL((gs_layout<T, 1, IN>), g, dim3(256), 0, st, grid, lay, (int)p.dims[0],
                           (int)p.dims[1], Wp, ntiles);
    if (IN)
        hipLaunchKernelGGL((gs_bottom_row<T>), dim3((unsigned)((p.dims[1] + 255) / 256)), dim3(256),
                           0, st, grid, lay, (int)p.dims[0], (int)p.dims[1], bands_of(p), Wp);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gs3d(const Problem& p, void* work, const void* coeffs, int sweeps,
                       hipStream_t st);
size_t gs3d_layout_bytes(const Problem& p);
hipError_t gs3d_layout(const Problem& p, void* grid, void* work, bool in, hipStream_t st);

size_t gs_state_bytes(const Problem& p) { return p.ndim != 2 ? 256 : state_bytes(p); }

size_t gs_work_bytes(const Problem& p) {
    // status word and block counters, then one ring per wave (8-byte slots)
    if (p.ndim == 1) return 256 + (size_t)kG1MaxWaves * kG1Ring * kG1Block * 8;
    if (p.ndim == 3) return 256 + gs3d_layout_bytes(p);  // status word, plane-major layout
    // nb bands and one slot for the bottom border row
    const size_t lay = (size_t)(bands_of(p) + 1) * (size_t)layout_width(p) * kRows * p.elem_bytes();
    return state_bytes(p) + lay;
}

hipError_t gs_layout_in(const Problem& p, const void* grid, void* work, hipStream_t st) {
    if (p.ndim == 1) return hipSuccess;  // the 1D kernel works on the grid itself
    if (p.ndim == 3) return gs3d_layout(p, (void*)grid, work, true, st);
    if (p.dtype == TVS_F64) return layout_t<double, true>(p, (double*)grid, work, st);
    return layout_t<float, true>(p, (float*)grid, work, st);
}

hipError_t gs_layout_out(const Problem& p, void* grid, void* work, hipStream_t st) {
    if (p.ndim == 1) return hipSuccess;
    if (p.ndim == 3) return gs3d_layout(p, grid, work, false, st);
    if (p.dtype == TVS_F64) return layout_t<double, false>(p, (double*)grid, work, st);
    return layout_t<float, false>(p, (float*)grid, work, st);
}

hipError_t launch_gs(const Problem& p, void* grid, const void* coeffs, int sweeps, void* work,
                     hipStream_t st) {
    if (p.ndim == 3) return launch_gs3d(p, work, coeffs, sweeps, st);
    if (p.ndim == 1) {
        if (sweeps < 1 || sweeps > 64 * kG1MaxWaves || p.dims[0] < 3) return hipErrorInvalidValue;
        const int waves = (sweeps + 63) / 64;
        const int n = (int)p.dims[0];
        int* w = (int*)work;
        int* prog = w + 16;
        void* ring = (char*)work + 256;
        hipLaunchKernelGGL(gs1d_reset, dim3(1), dim3(64), 0, st, prog, waves);
        if (p.dtype == TVS_F64)
            hipLaunchKernelGGL((gs1d_mc<double>), dim3((unsigned)waves), dim3(64), 0, st,
                               (double*)grid, n, sweeps, *(const Coeffs<double>*)coeffs,
                               (double*)ring, prog, w + 1);
        else
            hipLaunchKernelGGL((gs1d_mc<float>), dim3((unsigned)waves), dim3(64), 0, st,
                               (float*)grid, n, sweeps, *(const Coeffs<float>*)coeffs,
                               (float*)ring, prog, w + 1);
        return hipGetLastError();
    }
    if (p.dtype == TVS_F64)
        return launch_gs_t<double>(p, (double*)grid, *(const Coeffs<double>*)coeffs, sweeps, work,
                                   st);
    return launch_gs_t<float>(p, (float*)grid, *(const Coeffs<float>*)coeffs, sweeps, work, st);
}

hipError_t gs_read_status(const void* work, int* status, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(status, (const int*)work + 1, sizeof(int),
                                  hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

}  // namespace tvs
