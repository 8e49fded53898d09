/* Stencil oracle -- test infrastructure only (see oracle.c). */
#ifndef STENCIL_ORACLE_H
#define STENCIL_ORACLE_H
#include <stdint.h>

#define ORACLE_STAR 0
#define ORACLE_BOX 1
#define ORACLE_JACOBI 0
#define ORACLE_GAUSS_SEIDEL 1
#define ORACLE_DIRICHLET 0
#define ORACLE_PERIODIC 1

/* Canonical offsets (lexicographic, axis 0 most significant) as npoints rows
 * of ndim ints.  Returns the number of points, or a negative error code. */
int oracle_offsets(int ndim, int shape, int npoints, int *offsets_out);
/* Longest common subsequence table from a boundary row (n+1) and column
 * (col[1..m]) to the last row and column (0 = ok); see oracle.c. */
int oracle_lcs(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n, int32_t *row,
               int32_t *col);
/* Game of Life B2S23 on an n0 x n1 int32 board, T steps in place (0 = ok). */
int oracle_life(int64_t n0, int64_t n1, int boundary, int64_t T, int32_t *u);

/* T steps of the naive sweep on grid (C order, dims[0] slowest), in place.
 * Returns 0, or -1 bad argument, -2 point count inconsistent with the shape,
 * -3 an extent smaller than 2r+1, -4 Gauss-Seidel with periodic boundary,
 * -5 out of memory. */
int oracle_sweep_f64(int ndim, const int64_t *dims, int shape, int npoints, int dependence,
                     int boundary, const double *coeffs, int64_t T, double *grid);
int oracle_sweep_f32(int ndim, const int64_t *dims, int shape, int npoints, int dependence,
                     int boundary, const float *coeffs, int64_t T, float *grid);
/* Variable-coefficient Jacobi sweep (Section 3.4: LCS treats one sequence as
 * a coefficient that varies along the space axis): the weight of offset q at
 * the point with C-order index i is weights[q * N + i], N = prod(dims), the
 * same at every step.  Otherwise as oracle_sweep_*. */
int oracle_sweep_f64_varcoef(int ndim, const int64_t *dims, int shape, int npoints, int boundary,
                             const double *weights, int64_t T, double *grid);
int oracle_sweep_f32_varcoef(int ndim, const int64_t *dims, int shape, int npoints, int boundary,
                             const float *weights, int64_t T, float *grid);
#endif
