/*
 * Stencil oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, single-threaded, deliberately slow CPU implementation of the
 * time-iterated stencil sweep that the HIP library computes.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg use it; the
 * product path never calls, links or loads it.  It shares no code with the
 * HIP library.
 *
 * What it computes (Section 1 of the paper, the problem statement, and the
 * scalar 1D3P Jacobi code of Algorithm 1 in Section 2.1; Gauss-Seidel as
 * described in Section 3.4 "Gauss-Seidel stencils"):
 *
 *   - a regular d-dimensional grid u (d = 1, 2, 3), C order (axis 0 slowest);
 *   - a stencil of P points given by its shape (star or box) and radius r,
 *     P = 2*d*r + 1 (star) or (2r+1)^d (box);
 *   - the naive (d+1)-loop sweep: the outermost loop runs over time, the
 *     inner loops over the grid points in lexicographic order;
 *   - each point update is the weighted sum of its P neighbours,
 *       acc = c[0]*v[0];  acc = acc + c[q]*v[q]  for q = 1 .. P-1,
 *     with the offsets in canonical order: lexicographic over the offset
 *     vector, axis 0 most significant.  Every product and every sum is a
 *     separately rounded IEEE operation (this file must be compiled with
 *     -ffp-contract=off and without fast-math);
 *   - Jacobi: every update of step t+1 reads step-t values (a second buffer);
 *   - Gauss-Seidel: a single array updated in place in lexicographic order,
 *     so neighbours that come earlier in that order contribute their newest
 *     (this step's) value and the centre and later neighbours their previous
 *     one;
 *   - constant (Dirichlet) boundary: the outer r layers of every axis are
 *     part of the array, never written, and read as fixed values;
 *     periodic boundary: every point is updated and neighbour indices wrap.
 *
 * The FP32 entry points repeat the same loops in single precision (storage,
 * coefficients and arithmetic all float, same operation order).  They exist so
 * that the single-precision GPU path, which follows the same operation order,
 * can be checked bit for bit; the reference result for error statements is
 * the FP64 sweep.
 *
 * Pinned by tests that do not use this file's arithmetic: exact rational
 * brute force (Jacobi iteration matrix, Gauss-Seidel triangular solve),
 * Fourier and sine eigenmodes, the binomial closed form of the 1D 3-point
 * smoother, constant fields, fixed borders, translation invariance,
 * composition, the maximum principle, and the Gauss-Seidel/Jacobi
 * convergence factors of the discrete Laplacian.  The Game of Life sweep
 * (below) is pinned by boards whose next state is derived by counting
 * neighbours by hand, and by its invariants (fixed border, the square's
 * symmetries, translation on the torus, composition).  The LCS table is
 * pinned by brute force over all subsequences of short strings, a textbook
 * example, symmetry, and the chaining of rectangles through the wavefront
 * arrays.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define MAXD 3
#define MAXP 343 /* (2*3+1)^3: radius up to 3 in 3D */

/* Canonical offset list.  Returns P, or a negative value on bad input.  The
 * offsets are written as P rows of MAXD ints: row q holds (d0, d1, d2) padded
 * with zeros on the right for ndim < 3. */
static int canonical_offsets(int ndim, int shape, int npts, int *r_out, int offs[][MAXD])
{
    if (ndim < 1 || ndim > MAXD) return -1;
    int r = -1;
    for (int cand = 1; cand <= 3; ++cand) {
        int p = 1;
        if (shape == ORACLE_STAR) p = 2 * ndim * cand + 1;
        else if (shape == ORACLE_BOX) { for (int a = 0; a < ndim; ++a) p *= 2 * cand + 1; }
        else return -1;
        if (p == npts) { r = cand; break; }
    }
    if (r < 0) return -2;
    int side = 2 * r + 1, total = 1;
    for (int a = 0; a < ndim; ++a) total *= side;
    int P = 0;
    /* enumerate {-r..r}^ndim lexicographically, axis 0 most significant */
    for (int lin = 0; lin < total; ++lin) {
        int d[MAXD] = {0, 0, 0};
        int rem = lin, nonzero = 0;
        for (int a = ndim - 1; a >= 0; --a) {
            d[a] = rem % side - r;
            rem /= side;
            if (d[a] != 0) ++nonzero;
        }
        if (shape == ORACLE_STAR && nonzero > 1) continue;
        for (int a = 0; a < MAXD; ++a) offs[P][a] = d[a];
        ++P;
    }
    *r_out = r;
    return P;
}

int oracle_offsets(int ndim, int shape, int npoints, int *offsets_out)
{
    int offs[MAXP][MAXD];
    int r = 0;
    int P = canonical_offsets(ndim, shape, npoints, &r, offs);
    if (P < 0) return P;
    for (int q = 0; q < P; ++q)
        for (int a = 0; a < ndim; ++a) offsets_out[q * ndim + a] = offs[q][a];
    return P;
}

/* Periodic index: |i| stays within one extent of the range because r < n. */
static int64_t wrap(int64_t i, int64_t n)
{
    if (i < 0) return i + n;
    if (i >= n) return i - n;
    return i;
}

/* Shared argument checks; fills the padded 3-axis extents. */
static int prepare(int ndim, const int64_t *dims, int shape, int npts, int dependence,
                   int boundary, int64_t T, int *r, int offs[][MAXD], int64_t n[MAXD])
{
    if (!dims || T < 0) return -1;
    if (dependence != ORACLE_JACOBI && dependence != ORACLE_GAUSS_SEIDEL) return -1;
    if (boundary != ORACLE_DIRICHLET && boundary != ORACLE_PERIODIC) return -1;
    int P = canonical_offsets(ndim, shape, npts, r, offs);
    if (P < 0) return P;
    for (int a = 0; a < MAXD; ++a) n[a] = 1;
    for (int a = 0; a < ndim; ++a) {
        if (dims[a] < 2 * (int64_t)(*r) + 1) return -3;
        n[a] = dims[a];
    }
    return P;
}

/*
 * The sweep, written once as a macro over the scalar type so that the FP64
 * and FP32 variants are textually identical.  The grid is viewed as 3D with
 * leading unit axes for ndim < 3; a unit axis has a single index and a zero
 * offset component, which leaves the lexicographic order unchanged.
 */
/* wts == NULL: the weights are coeffs[q] at every point; otherwise the weight
 * of offset q at the point with C-order index i is wts[q * N + i] (N grid
 * points), fixed over time -- a variable-coefficient stencil. */
#define DEFINE_SWEEP(NAME, REAL)                                                          \
static int NAME##_impl(int ndim, const int64_t *dims, int shape, int npoints,            \
                       int dependence, int boundary, const REAL *coeffs, const REAL *wts, \
                       int64_t T, REAL *grid)                                             \
{                                                                                         \
    int r = 0;                                                                            \
    int offs[MAXP][MAXD];                                                                 \
    int64_t n[MAXD];                                                                      \
    if ((!coeffs && !wts) || !grid) return -1;                                            \
    int P = prepare(ndim, dims, shape, npoints, dependence, boundary, T, &r, offs, n);   \
    if (P < 0) return P;                                                                  \
    if (dependence == ORACLE_GAUSS_SEIDEL && boundary == ORACLE_PERIODIC) return -4;      \
    /* place the real axes last: axis a of the problem is axis (MAXD-ndim+a) here */      \
    int64_t ext[MAXD];                                                                    \
    int o[MAXP][MAXD];                                                                    \
    for (int a = 0; a < MAXD; ++a) ext[a] = 1;                                            \
    for (int a = 0; a < ndim; ++a) ext[MAXD - ndim + a] = n[a];                           \
    for (int q = 0; q < P; ++q) {                                                         \
        for (int a = 0; a < MAXD; ++a) o[q][a] = 0;                                       \
        for (int a = 0; a < ndim; ++a) o[q][MAXD - ndim + a] = offs[q][a];                \
    }                                                                                     \
    int64_t lo[MAXD], hi[MAXD];                                                           \
    for (int a = 0; a < MAXD; ++a) {                                                      \
        int real_axis = a >= MAXD - ndim;                                                 \
        lo[a] = (real_axis && boundary == ORACLE_DIRICHLET) ? r : 0;                      \
        hi[a] = (real_axis && boundary == ORACLE_DIRICHLET) ? ext[a] - r : ext[a];        \
    }                                                                                     \
    int64_t total = ext[0] * ext[1] * ext[2];                                             \
    REAL *src = grid, *dst = grid, *spare = NULL;                                         \
    if (dependence == ORACLE_JACOBI) {                                                    \
        spare = (REAL *)malloc((size_t)total * sizeof(REAL));                             \
        if (!spare) return -5;                                                            \
        memcpy(spare, grid, (size_t)total * sizeof(REAL)); /* fixed border values */      \
        dst = spare;                                                                      \
    }                                                                                     \
    /* linear distance of each neighbour (used where no index wraps) */                \
    int64_t lin[MAXP];                                                                    \
    for (int q = 0; q < P; ++q)                                                           \
        lin[q] = ((int64_t)o[q][0] * ext[1] + o[q][1]) * ext[2] + o[q][2];                \
    for (int64_t t = 0; t < T; ++t) {                                                     \
        for (int64_t i = lo[0]; i < hi[0]; ++i)                                           \
            for (int64_t j = lo[1]; j < hi[1]; ++j)                                       \
                for (int64_t k = lo[2]; k < hi[2]; ++k) {                                 \
                    int64_t at = (i * ext[1] + j) * ext[2] + k;                           \
                    REAL acc = 0;                                                         \
                    for (int q = 0; q < P; ++q) {                                         \
                        REAL v;                                                           \
                        if (boundary == ORACLE_DIRICHLET) {                               \
                            v = src[at + lin[q]];                                         \
                        } else {                                                          \
                            int64_t ii = wrap(i + o[q][0], ext[0]);                       \
                            int64_t jj = wrap(j + o[q][1], ext[1]);                       \
                            int64_t kk = wrap(k + o[q][2], ext[2]);                       \
                            v = src[(ii * ext[1] + jj) * ext[2] + kk];                    \
                        }                                                                 \
                        REAL wq = wts ? wts[(int64_t)q * total + at] : coeffs[q];         \
                        REAL term = wq * v;                                               \
                        acc = (q == 0) ? term : acc + term;                               \
                    }                                                                     \
                    dst[at] = acc;                                                        \
                }                                                                         \
        if (dependence == ORACLE_JACOBI) { REAL *tmp = src; src = dst; dst = tmp; }       \
    }                                                                                     \
    if (dependence == ORACLE_JACOBI) {                                                    \
        if (src != grid) memcpy(grid, src, (size_t)total * sizeof(REAL));                 \
        free(spare);                                                                      \
    }                                                                                     \
    return 0;                                                                             \
}                                                                                         \
int NAME(int ndim, const int64_t *dims, int shape, int npoints, int dependence,           \
         int boundary, const REAL *coeffs, int64_t T, REAL *grid)                         \
{                                                                                         \
    if (!coeffs) return -1;                                                               \
    return NAME##_impl(ndim, dims, shape, npoints, dependence, boundary, coeffs, NULL, T, \
                       grid);                                                             \
}                                                                                         \
int NAME##_varcoef(int ndim, const int64_t *dims, int shape, int npoints, int boundary,  \
                   const REAL *weights, int64_t T, REAL *grid)                            \
{                                                                                         \
    if (!weights) return -1;                                                              \
    return NAME##_impl(ndim, dims, shape, npoints, ORACLE_JACOBI, boundary, NULL,        \
                       weights, T, grid);                                                 \
}

DEFINE_SWEEP(oracle_sweep_f64, double)
DEFINE_SWEEP(oracle_sweep_f32, float)

/*
 * Game of Life, variant B2S23 -- the rule the paper adopts for its Life
 * stencil (Section 3.4, "Game of life"): a 2D 9-point box stencil on integer
 * cells where a dead cell becomes live when exactly 2 of its 8 neighbours are
 * live and a live cell stays live when 2 or 3 are.  Cells are int32; a cell
 * is live when it is non-zero, and its neighbour count is the sum of its 8
 * neighbours' values (the number of live neighbours on a 0/1 board).  The new
 * value is 1 or 0.  Jacobi: every cell of step t+1 reads step-t values.
 * Dirichlet: the outer layer never changes; periodic: indices wrap.
 */
int oracle_life(int64_t n0, int64_t n1, int boundary, int64_t T, int32_t *u)
{
    if (n0 < 3 || n1 < 3 || T < 0 || !u) return -1;
    if (boundary != 0 && boundary != 1) return -1;
    const int64_t n = n0 * n1;
    int32_t *v = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!v) return -2;
    int32_t *cur = u, *nxt = v;
    for (int64_t t = 0; t < T; ++t) {
        memcpy(nxt, cur, (size_t)n * sizeof(int32_t));
        const int64_t lo = boundary == 1 ? 0 : 1;
        for (int64_t i = lo; i < n0 - lo; ++i) {
            for (int64_t j = lo; j < n1 - lo; ++j) {
                int64_t s = 0;
                for (int di = -1; di <= 1; ++di) {
                    for (int dj = -1; dj <= 1; ++dj) {
                        if (di == 0 && dj == 0) continue;
                        const int64_t ii = wrap(i + di, n0), jj = wrap(j + dj, n1);
                        s += cur[ii * n1 + jj];
                    }
                }
                const int32_t c = cur[i * n1 + j];
                nxt[i * n1 + j] = (s == 2 || (c != 0 && s == 3)) ? 1 : 0;
            }
        }
        int32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    if (cur != u) memcpy(u, cur, (size_t)n * sizeof(int32_t));
    free(v);
    return 0;
}

/*
 * Longest common subsequence (Section 3.4, "Longest common subsequence"):
 * the dynamic program over the iteration space x = 1..m (time), y = 1..n
 * (space), where lcs[x][y] is the length of a longest common subsequence of
 * the prefixes a[1..x] and b[1..y]:
 *   lcs[x][y] = lcs[x-1][y-1] + 1              if a[x] == b[y],
 *             = max(lcs[x-1][y], lcs[x][y-1])  otherwise.
 * The run starts from a boundary row lcs[0][0..n] (row, n+1 values) and a
 * boundary column lcs[1..m][0] (col[1..m]; col[0] is not read), and returns
 * the last row lcs[m][0..n] in row and the last column lcs[0..m][n] in col:
 * the two wavefront arrays through which rectangles of the iteration space
 * are chained.  With all-zero boundaries, lcs[m][n] is the LCS length.
 * Sequences are byte strings; a[1..m] is a[0..m-1] in memory.  Row by row,
 * one row of storage.  Returns 0, -1 on a bad argument, -5 out of memory.
 */
int oracle_lcs(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n, int32_t *row,
               int32_t *col)
{
    if (m < 0 || n < 0 || !row || !col || (m > 0 && !a) || (n > 0 && !b)) return -1;
    int32_t *prev = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t *cur = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return -5;
    }
    memcpy(prev, row, (size_t)(n + 1) * sizeof(int32_t));
    col[0] = prev[n];  /* lcs[0][n] */
    for (int64_t x = 1; x <= m; ++x) {
        cur[0] = col[x];  /* lcs[x][0], the boundary column */
        for (int64_t y = 1; y <= n; ++y) {
            if (a[x - 1] == b[y - 1]) {
                cur[y] = prev[y - 1] + 1;
            } else {
                cur[y] = prev[y] > cur[y - 1] ? prev[y] : cur[y - 1];
            }
        }
        col[x] = cur[n];
        int32_t *tmp = prev;
        prev = cur;
        cur = tmp;
    }
    memcpy(row, prev, (size_t)(n + 1) * sizeof(int32_t));
    free(prev);
    free(cur);
    return 0;
}
