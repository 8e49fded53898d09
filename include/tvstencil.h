/*
 * tvstencil -- time-skewed temporal stencil sweeps for AMD Instinct MI355X
 * (gfx950).  C ABI.
 *
 * The problem (Section 1 of "Temporal Vectorization for Stencils"): a
 * time-iterated update of a regular d-dimensional grid (d = 1, 2, 3) by a
 * stencil that is classified by its number of points ("order"), its shape
 * (star or box), its dependence type (Jacobi or Gauss-Seidel) and its
 * boundary condition (constant or periodic).  The naive form is d+1 nested
 * loops with time outermost (Section 1; Algorithm 1 in Section 2.1 for the
 * 1D 3-point case).
 *
 * Definition of one step, which every entry point below reproduces exactly:
 *   - the grid is dense, C order: axis 0 slowest, the last axis contiguous;
 *     dims[] are full storage extents;
 *   - the stencil's P offsets are listed in canonical order: lexicographic
 *     over the offset vector with axis 0 most significant (2D 5-point:
 *     (-1,0), (0,-1), (0,0), (0,1), (1,0));
 *   - a point update is acc = c[0]*v[0], then acc = acc + c[q]*v[q] for
 *     q = 1..P-1, each product and sum rounded separately (no fused
 *     multiply-add, no reassociation), in the grid's precision;
 *   - Jacobi: all updates of step t+1 read step-t values;
 *   - Gauss-Seidel: one array updated in place in lexicographic point order,
 *     so neighbours that precede a point contribute their newest value
 *     (Section 3.4, "Gauss-Seidel stencils");
 *   - constant (Dirichlet) boundary: the outer r layers of every axis are
 *     never written and are read as fixed values; periodic: every point is
 *     updated and indices wrap.
 * The kernels reorder whole point updates only (time skewing, Section 3.2),
 * never the arithmetic inside one, so FP64 results are bit-identical to the
 * naive loops, and FP32 results are bit-identical to the naive loops run in
 * FP32, for every tuning.
 *
 * Conventions for every function:
 *   - returns TVS_OK (0) or a negative TVS_E_* code; nothing throws or aborts
 *     across the ABI; stencil_last_error() gives a thread-local message;
 *   - argument errors are reported synchronously; device work is enqueued
 *     asynchronously on the given HIP stream (NULL = the null stream);
 *   - device pointers are plain hipMalloc'd (or torch) allocations on the
 *     current device; host pointers are read during the call only;
 *   - the library never retains a caller's pointer after the stream work of
 *     the call has completed.
 */
#ifndef TVSTENCIL_H
#define TVSTENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define TVS_OK 0
#define TVS_E_INVALID (-1)     /* null pointer, bad enum, T < 0, bad tuning */
#define TVS_E_SHAPE (-2)       /* ndim not 1..3, an extent < 2r+1, size overflow */
#define TVS_E_ORDER (-3)       /* point count inconsistent with ndim and shape */
#define TVS_E_UNSUPPORTED (-4) /* e.g. periodic Gauss-Seidel, the 3D radius-3 box */
#define TVS_E_NOMEM (-5)       /* device or host allocation failed */
#define TVS_E_DEVICE (-6)      /* a HIP call failed or a kernel reported abort */
#define TVS_E_BUSY (-7)        /* server: budget or queue full */
#define TVS_E_NOTFOUND (-8)    /* server: unknown request id */

/* ---- enums ------------------------------------------------------------- */
#define TVS_F32 0
#define TVS_F64 1
#define TVS_I32 2 /* int32 cells: Game of Life plans only (stencil_plan_life) */
#define TVS_STAR 0
#define TVS_BOX 1
#define TVS_JACOBI 0
#define TVS_GAUSS_SEIDEL 1
#define TVS_DIRICHLET 0
#define TVS_PERIODIC 1

/* update rules: the weighted sum defined above, or Game of Life B2S23 */
#define TVS_RULE_WEIGHTED 0
#define TVS_RULE_LIFE 1

/* execution methods a plan can use */
#define TVS_METHOD_PLAIN 0 /* one time step per kernel launch (the baseline) */
#define TVS_METHOD_TSTP 1  /* time-skewed temporal pipeline, k steps per band */

typedef struct tvs_plan tvs_plan;

typedef struct tvs_plan_info {
    int ndim;
    int64_t dims[3];
    int dtype, shape, order, dependence, boundary;
    int radius;        /* r, derived from (ndim, shape, order) */
    int method;        /* TVS_METHOD_* */
    int k;             /* time-tile depth: steps per band (levels per pipeline) */
    int s;             /* skew: stream positions between successive levels */
    int tile_w;        /* non-stream tile extent in points, halo included
                          (2D: columns; 3D: columns of the inner tile) */
    int tile_h;        /* 3D: rows of the inner tile; 1 otherwise */
    int tile_l;        /* stream-axis segment length (output points) */
    int lane_c;        /* consecutive points per lane along the last axis */
    int lanemap;       /* 0 = successive levels in successive lanes,
                          1 = successive levels in successive waves */
    size_t scratch_bytes; /* device memory the plan owns */
    int pl;            /* 1D: lanes per pipeline (16 or 64) */
    int kern;          /* kernel kind: always 0 (LDS level planes) */
    char tuning[160];  /* the schedule as a tuning string that stencil_plan accepts */
    int rule;          /* TVS_RULE_WEIGHTED or TVS_RULE_LIFE */
    char varcoef_tuning[160]; /* the schedule stencil_run_varcoef runs (2D/3D: at most
                                 4 points per lane; without a tuning string, 2D radius 1
                                 takes its own tile and depth) */
} tvs_plan_info;

/*
 * Create a plan: validate the problem and choose how to run it.
 *   ndim        1, 2 or 3
 *   dims        ndim storage extents (halo/border included), each >= 2r+1
 *   dtype       TVS_F32 or TVS_F64 (storage and arithmetic precision)
 *   shape       TVS_STAR or TVS_BOX
 *   order       number of stencil points P (star: 2*ndim*r+1, box: (2r+1)^ndim);
 *               stars and boxes of radius 1..3 with at most 125 points
 *               (every one but the 3D radius-3 box, 343 points); boxes of
 *               more than 27 points (2D radius 3, 3D radius 2) run plain
 *               steps; Gauss-Seidel: radius 1 only
 *   dependence  TVS_JACOBI or TVS_GAUSS_SEIDEL
 *   boundary    TVS_DIRICHLET or TVS_PERIODIC (Gauss-Seidel: Dirichlet only)
 *   tuning      NULL: the tuned default (autotune cache, else a model-based
 *               choice); otherwise "key=value" pairs separated by commas:
 *               method=plain|tstp, k=, s=, w=, h=, l=, c=, lanemap=, pl=, kern=0
 * The plan is created without touching the device; device scratch (the
 * Jacobi second buffer) is allocated at the first run and freed by
 * stencil_plan_destroy.  *out is set only on success.
 */
int stencil_plan(tvs_plan **out, int ndim, const int64_t *dims, int dtype, int shape, int order,
                 int dependence, int boundary, const char *tuning);

/*
 * Create a Game of Life plan: the B2S23 cellular automaton, one of the
 * stencils the paper evaluates (Section 3.4 and Table 1, "Life": a 2D
 * 9-point box stencil on integer cells).  One step, Jacobi-style (every cell
 * of step t+1 reads step-t values):
 *   s   = the sum of the values of the 8 neighbours (axis 0 and axis 1 offsets
 *         in {-1, 0, 1}, the centre excluded), in 32-bit integer arithmetic;
 *   new = 1 if s == 2, or if the cell is non-zero and s == 3; else 0.
 * On a 0/1 board s is the number of live neighbours: a dead cell is born with
 * exactly 2 of them and a live cell survives with 2 or 3.  Boards whose
 * values lie within +-2^27 (0/1 boards in particular) never overflow the sum,
 * so the result is that of the definition with exact integer sums.
 *   ndim      must be 2
 *   dims      2 storage extents, each >= 3
 *   boundary  TVS_DIRICHLET: the outer layer of cells is never written (it
 *             keeps any values it holds); TVS_PERIODIC: indices wrap
 *   tuning    as for stencil_plan (2D Jacobi keys)
 * The plan has dtype TVS_I32, shape TVS_BOX, order 9, dependence TVS_JACOBI
 * and rule TVS_RULE_LIFE.  stencil_run and stencil_tune take such a plan
 * with coeffs NULL (any coeffs given are ignored); the grid is prod(dims)
 * int32 values.  stencil_batch_run and the server do not take Life plans
 * (TVS_E_UNSUPPORTED), and stencil_plan and stencil_run_simple reject
 * TVS_I32 (TVS_E_INVALID).
 */
int stencil_plan_life(tvs_plan **out, int ndim, const int64_t *dims, int boundary,
                      const char *tuning);

/* Fill *info with the plan's problem and chosen schedule. */
int stencil_plan_info(const tvs_plan *plan, tvs_plan_info *info);

/* Free the plan and everything it owns.  Waits for the device first.  NULL is a no-op. */
int stencil_plan_destroy(tvs_plan *plan);

/*
 * Advance grid by T steps.
 *   grid    device pointer, prod(dims) elements of the plan's dtype, C order;
 *           input at step 0, output at step T (in place from the caller's
 *           view; Jacobi uses the plan's second buffer internally)
 *   coeffs  host array of P doubles in canonical offset order; rounded to
 *           FP32 (nearest even) for TVS_F32 plans; copied during the call;
 *           NULL (and ignored) for Life plans
 *   T       >= 0; T = 0 enqueues nothing
 *   stream  hipStream_t or NULL
 * One plan runs on one stream at a time; distinct plans may run concurrently.
 * Gauss-Seidel runs wait for their producers with bounded spins.  A wait that
 * expires makes that run's result (and that of every later run of the plan,
 * until it is reported) invalid.  The device work is asynchronous, so the
 * abort is reported (TVS_E_DEVICE, nothing enqueued) by the first later
 * stencil_run or stencil_batch_run of the plan that finds the earlier run
 * complete, or by stencil_plan_check, which waits for it.  Reporting clears
 * it.
 */
int stencil_run(tvs_plan *plan, void *grid, const double *coeffs, int64_t T, void *stream);

/*
 * Wait until the plan's last Gauss-Seidel run has completed and report
 * whether any of its launches (or of earlier unreported runs) aborted:
 * TVS_OK, or TVS_E_DEVICE (and the abort is cleared).  Jacobi and Life plans,
 * and plans that have not run, return TVS_OK at once.  Synchronizes the host
 * with that run; it enqueues nothing.
 */
int stencil_plan_check(tvs_plan *plan);

/*
 * Advance grid by T Jacobi steps of a variable-coefficient stencil: the
 * weight of offset q at the point with C-order index i is weights[q * N + i]
 * (N = prod(dims), offsets in canonical order), the same at every step
 * (Section 3.4 treats LCS's sequence B as such a coefficient, one that varies
 * along the space axis).  Each update is w_0(i)*v_0 + w_1(i)*v_1 + ... in
 * the order and rounding stated above.
 *   weights  device, P * N elements of the plan's dtype (F32 or F64); read
 *            only, not retained
 * Jacobi plans only (Gauss-Seidel: TVS_E_UNSUPPORTED; Life: TVS_E_INVALID).
 * Plans with a time-skewed schedule run bands of k levels: 1D with the
 * weights staged in LDS (up to 64 levels), 2D and 3D (radius 1 and 2, at
 * most 27 points) with 4 points per lane: 2D radius 1 with each point row's
 * weights staged in an LDS ring and, without a tuning string, its own tile
 * and depth (stencil_plan_info's varcoef_tuning), the others on the plan's
 * tile shape with each weight read by the level that forms its term.  3D
 * radius 3, boxes of more than 27 points and plain schedules run one step
 * per launch.
 */
int stencil_run_varcoef(tvs_plan *plan, void *grid, const void *weights, int64_t T, void *stream);

/*
 * One-call form: plans (through an internal cache keyed by the problem and the
 * current device) and runs; arguments as in stencil_plan and stencil_run.
 * Calls for the same problem share one cached plan and its scratch: each call
 * holds the plan while it enqueues, and its stream first waits for the
 * previous call's work, so calls from several threads or on several streams
 * are safe (and run one after the other on the device).
 */
int stencil_run_simple(void *grid, int ndim, const int64_t *dims, int dtype, const double *coeffs,
                       int shape, int order, int dependence, int boundary, int64_t T,
                       void *stream);

/*
 * Run n independent problems on one stream.  The Jacobi members of one
 * kernel variant (precision, dimension, shape, boundary, points per lane) run
 * in one persistent launch: every band of every such grid is cut into tiles,
 * workgroups take tiles from a work list in band order, and a tile waits
 * only until its grid's previous band is complete.  Each member keeps its
 * plan's schedule (depth, tile shape, segment length, lane map; a plan whose
 * schedule the batch kernels cannot take, e.g. plain steps, runs a default
 * time-skewed one).  Gauss-Seidel plans run through their own persistent
 * kernel, next to the Jacobi launches.  grids[i], coeffs[i], T[i] as in
 * stencil_run.  A plan or a grid may appear at most once among the members
 * with T[i] > 0 (TVS_E_INVALID): members run at the same time.  Radius > 1
 * and Game of Life plans are not taken (TVS_E_UNSUPPORTED).  Every result is
 * bit-identical to stencil_run of the same problem alone.  The launch
 * sequence is captured once in a hipGraph per distinct batch layout and
 * replayed.  A persistent launch whose bounded wait expires (results
 * invalid) is reported by the next call (TVS_E_DEVICE).
 */
int stencil_batch_run(int n, tvs_plan *const *plans, void *const *grids,
                      const double *const *coeffs, const int64_t *T, void *stream);

/*
 * Autotune: time candidate schedules for this plan's problem on `grid`
 * (contents are restored afterwards) over T_probe steps -- or two bands of
 * the candidate's depth if that is longer; candidates are compared per
 * step -- keep the fastest,
 * record it in the tuning cache (path from TVS_TUNE_CACHE, if set), and
 * switch the plan to it.  Candidates that do not produce the same bits as
 * the first one are rejected (TVS_E_DEVICE).  best (may be NULL) receives
 * the winning tuning string.
 */
int stencil_tune(tvs_plan *plan, void *grid, const double *coeffs, int64_t T_probe,
                 void *stream, char *best, size_t best_len);

/* ---- longest common subsequence ------------------------------------------ */
/*
 * The LCS dynamic program as a 1D Gauss-Seidel-like stencil (Section 3.4,
 * "Longest common subsequence"): with x = 1..m as the time axis and
 * y = 1..n as the space axis,
 *   L[x][y] = L[x-1][y-1] + 1            if A[x] == B[y],
 *           = max(L[x-1][y], L[x][y-1])  otherwise,
 * where A[x] = a[x-1] and B[y] = b[y-1] are bytes.  A run starts from a
 * boundary row L[0][0..n] and a boundary column L[1..m][0] and returns the
 * last row L[m][0..n] and the last column L[0..m][n]: the wavefront arrays
 * through which rectangles of the iteration space are chained.  With zero
 * boundaries, L[m][n] is the length of a longest common subsequence of A and
 * B (and L[m][y], L[x][n] those of A and B[1..y], A[1..x] and B).
 */
typedef struct tvs_lcs tvs_lcs;

/* Plan a run for lengths m, n (each 0 .. 2^30).  tuning: NULL, or
 * comma-separated "w=W" (tile width in columns, a multiple of 64 in 64..4096,
 * default 1024) and "r=R" (tile height in rows, a multiple of 64 in 64..1024,
 * default 256: one wave per 64 rows); (R/64 + 1) x (W + 192) int32 values
 * must fit 160 KiB of LDS.  No device call; a corner array of ceil(n/W)
 * int32 values is allocated at the first run. */
int stencil_lcs_plan(tvs_lcs **out, int64_t m, int64_t n, const char *tuning);
/* The plan's tile width in columns and height in rows (TVS_E_INVALID for NULL). */
int stencil_lcs_tile_width(const tvs_lcs *plan);
int stencil_lcs_tile_rows(const tvs_lcs *plan);
/*
 * Enqueue the run on stream (NULL = the null stream).
 *   a    device, m bytes (may be NULL when m = 0)
 *   b    device, n bytes (may be NULL when n = 0)
 *   row  device int32[n+1]: in L[0][y]; out L[m][y], y = 0..n
 *   col  device int32[m+1]: in col[x] = L[x][0] for x = 1..m (col[0] is not
 *        read); out col[x] = L[x][n], x = 0..m
 * Values are int32; every L is the sum of a boundary value and at most
 * min(m, n), which must not overflow.  a, b, row and col must not overlap.
 * One plan runs on one stream at a time.
 */
int stencil_lcs_run(tvs_lcs *plan, const uint8_t *a, const uint8_t *b, int32_t *row,
                    int32_t *col, void *stream);
/*
 * stencil_lcs_run for callers that cannot allocate device memory (code under
 * hipGraph capture, serving loops, harnesses that forbid hipMalloc): the same
 * launches and results, with the per-tile-column corner array in a static
 * device array of 65536 int32 (256 KiB; every device the library runs on
 * holds one until the process ends) instead of memory the plan allocates.
 * The call allocates nothing and frees nothing.  Arguments as for
 * stencil_lcs_run.
 *   - the plan may have at most 65536 tile columns, ceil(n / w) <= 65536
 *     (n <= 67108864 with the default w = 1024); larger: TVS_E_SHAPE;
 *   - all calls on one device share that device's array and nothing in it
 *     needs to start at zero (each run writes every entry it reads first);
 *     calls that overlap on one device (on several streams, or from several
 *     threads without ordering) race on it and give invalid results.
 */
int stencil_lcs_run_noalloc(const tvs_lcs *plan, const uint8_t *a, const uint8_t *b,
                            int32_t *row, int32_t *col, void *stream);

/* Free the plan (waits for the device first).  NULL is a no-op. */
int stencil_lcs_destroy(tvs_lcs *plan);

/* ---- serving: continuous batching of stencil solves ----------------------- */
typedef struct tvs_server tvs_server;

typedef struct tvs_request {
    int ndim;
    int64_t dims[3];
    int dtype, shape, order, dependence, boundary;
    const double *coeffs; /* host, P doubles, copied at submit */
    int64_t T;
    const void *host_in;  /* host, prod(dims) elements, copied at submit */
} tvs_request;

typedef struct tvs_server_stats {
    uint64_t submitted, admitted, completed, rejected;
    uint64_t chunks;           /* persistent launches issued */
    uint64_t resident;         /* grids on the device now */
    size_t bytes_in_use;       /* device bytes held by resident grids */
    double busy_seconds;       /* device time of all chunks */
    double updates;            /* point updates completed */
} tvs_server_stats;

/*
 * Start a server on the current device.  hbm_budget: device bytes resident
 * grids may occupy (0 = 4 GiB); max_slots: grids resident at once (0 = 64);
 * chunk_steps: steps per grid per chunk (0 = 64).  A background thread admits
 * queued requests in arrival order whenever their footprint fits the budget
 * and a slot is free, advances every resident grid by up to chunk_steps per
 * chunk in one batched launch, and retires finished grids.
 */
int stencil_server_create(tvs_server **out, size_t hbm_budget, int max_slots, int chunk_steps);
/* Queue a request; *id identifies it.  TVS_E_BUSY if it can never fit the budget. */
int stencil_server_submit(tvs_server *srv, const tvs_request *req, uint64_t *id);
/* Non-blocking: *status = 1 done, 0 pending; on done copies the result to host_out
 * (prod(dims) elements) if not NULL and forgets the request.  Timestamps (seconds
 * on the server clock) are written to t_out[0..3] = arrival, admit, start, finish
 * if t_out is not NULL. */
int stencil_server_poll(tvs_server *srv, uint64_t id, int *status, void *host_out, double *t_out);
/* Blocking form of poll. */
int stencil_server_wait(tvs_server *srv, uint64_t id, void *host_out, double *t_out);
int stencil_server_stats(tvs_server *srv, tvs_server_stats *out);
/* Seconds on the server clock (monotonic, zero at create). */
double stencil_server_now(tvs_server *srv);
/* Stop the thread, drop pending work, free device memory. */
int stencil_server_destroy(tvs_server *srv);

/* Message for the last non-zero return on this thread ("" if none). */
const char *stencil_last_error(void);

/* Library version string. */
const char *stencil_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TVSTENCIL_H */
