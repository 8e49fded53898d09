// Kernel launchers shared between the HIP translation units.
#pragma once

#include "common.hpp"

namespace tvs {

// One plain Jacobi step in -> out (all points written; fixed borders copied).
hipError_t launch_plain_step(const Problem& p, const void* in, void* out, const void* coeffs,
                             hipStream_t st);

// Copy bytes device to device with a kernel (graph-capture friendly).
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);

// Geometry of one time-skewed band: derived from the schedule for a band of
// `k` levels.  Shared by the launcher, the batch kernel and the tuner.
struct BandGeom {
    int k = 1;           // levels in this band
    int W = 0, H = 1;    // tile extents (halo included) along the last axis / axis 1 (3D)
    int Wv = 0, Hv = 1;  // valid outputs per tile along those axes
    int Lv = 0;          // valid outputs per stream segment
    int C = 1;           // points per lane along the last axis
    int G = 0;           // lanes per level
    int NT = 0;          // threads per workgroup
    int ntx = 1, nty = 1, nseg = 1;  // tile counts
    int pl = 64;         // 1D: lanes per pipeline
    int lanemap = 0;
    int kern = 0;        // 0 = LDS level planes (the only kind)
    size_t lds_bytes = 0;
    int tiles_per_block = 1;
    int64_t tiles() const { return (int64_t)ntx * nty * nseg; }
    int64_t blocks() const { return (tiles() + tiles_per_block - 1) / tiles_per_block; }
};

// Fill geometry for a band of k levels; returns false if the schedule cannot
// run this band (thread or LDS limits).
bool band_geometry(const Problem& p, const Schedule& s, int k, BandGeom* g);

// One time-skewed band of g.k Jacobi steps in -> out.
hipError_t launch_tstp_band(const Problem& p, const BandGeom& g, const void* in, void* out,
                            const void* coeffs, hipStream_t st);

// The 2D/3D band kernel for radius 1..3 with constant weights (radius > 1)
// or variable coefficients (wts != nullptr: P weight planes of the grid's
// size, offset-major): geometry of a band of k levels (vc: for variable
// coefficients), and one band.
bool ndr_geometry(const Problem& p, const Schedule& s, int k, BandGeom* g, bool vc = false);
hipError_t launch_tstp_ndr(const Problem& p, const BandGeom& g, const void* in, void* out,
                           const void* coeffs, const void* wts, hipStream_t st);

// Gauss-Seidel.  `work` is device scratch of gs_work_bytes(p) bytes whose
// first gs_state_bytes(p) bytes are zero before its first launch.  A run is
// gs_layout_in (interior rows of grid -> band layout in work), launch_gs
// calls of up to 256 sweeps each (one persistent launch per call; the two
// border rows are read from grid), and gs_layout_out (band layout -> grid).
size_t gs_state_bytes(const Problem& p);
size_t gs_work_bytes(const Problem& p);
hipError_t gs_layout_in(const Problem& p, const void* grid, void* work, hipStream_t st);
hipError_t launch_gs(const Problem& p, void* grid, const void* coeffs, int sweeps, void* work,
                     hipStream_t st);
hipError_t gs_layout_out(const Problem& p, void* grid, void* work, hipStream_t st);
// Status word written by the Gauss-Seidel kernel (0 = ok) lives in `work`.
hipError_t gs_read_status(const void* work, int* status, hipStream_t st);

// True when every weight has the bit pattern of the first.  Only then may an
// interior tile form each value's product once and reuse it for every
// offset: weights that compare equal but differ in sign (-0.0 and +0.0)
// give products of different sign, and the canonical sum of those can be
// +0.0 where the shared product would give -0.0.
bool same_weight_bits(const double* c, int n);

// Whether the schedule's kernel exists for this problem.
bool tstp_supported(const Problem& p);

}  // namespace tvs
