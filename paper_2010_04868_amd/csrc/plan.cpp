// Host-side planning: problem validation, radius and legality, tuning
// strings and the model-based default schedule.  No device calls here, so a
// plan can be created (and its validation tested) on a machine without a GPU.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "kernels.hpp"
#include "plan.hpp"

namespace tvs {

static thread_local std::string g_last_error;

bool radius_supported(int ndim, int shape, int r);
size_t tstp1d_radius_lds_bytes(const Problem& p, int k, int Lv);

int set_error(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}
void clear_error() { g_last_error.clear(); }
const char* last_error() { return g_last_error.c_str(); }

// Radius from the point count, which Section 1 uses as a stencil's order:
// star P = 2*d*r + 1, box P = (2r+1)^d.
static int radius_of(int ndim, int shape, int order) {
    for (int r = 1; r <= 8; ++r) {
        int P = 1;
        if (shape == TVS_STAR) {
            P = 2 * ndim * r + 1;
        } else {
            for (int a = 0; a < ndim; ++a) P *= 2 * r + 1;
        }
        if (P == order) return r;
        if (P > order) break;
    }
    return -1;
}

int validate(Problem* pr, int ndim, const int64_t* dims, int dtype, int shape, int order,
             int dependence, int boundary) {
    if (!dims) return set_error(TVS_E_INVALID, "dims is NULL");
    if (ndim < 1 || ndim > 3) return set_error(TVS_E_SHAPE, "ndim must be 1, 2 or 3");
    if (dtype == TVS_I32)
        return set_error(TVS_E_INVALID, "int32 grids are Game of Life boards: use stencil_plan_life");
    if (dtype != TVS_F32 && dtype != TVS_F64) return set_error(TVS_E_INVALID, "bad dtype");
    if (shape != TVS_STAR && shape != TVS_BOX) return set_error(TVS_E_INVALID, "bad shape");
    if (dependence != TVS_JACOBI && dependence != TVS_GAUSS_SEIDEL)
        return set_error(TVS_E_INVALID, "bad dependence");
    if (boundary != TVS_DIRICHLET && boundary != TVS_PERIODIC)
        return set_error(TVS_E_INVALID, "bad boundary");
    const int r = radius_of(ndim, shape, order);
    if (r < 0)
        return set_error(TVS_E_ORDER, "order " + std::to_string(order) +
                                          " is not a star or box point count for ndim " +
                                          std::to_string(ndim));
    int64_t total = 1;
    for (int a = 0; a < ndim; ++a) {
        if (dims[a] < 2 * r + 1)
            return set_error(TVS_E_SHAPE, "extent " + std::to_string(dims[a]) + " of axis " +
                                              std::to_string(a) + " is below 2r+1");
        if (dims[a] > (int64_t)1 << 30)
            return set_error(TVS_E_SHAPE, "extent above 2^30");
        if (total > ((int64_t)1 << 40) / dims[a]) return set_error(TVS_E_SHAPE, "size overflow");
        total *= dims[a];
    }
    if (r != 1 && dependence == TVS_GAUSS_SEIDEL)
        return set_error(TVS_E_UNSUPPORTED, "Gauss-Seidel is implemented for radius 1");
    if (r != 1 && !radius_supported(ndim, shape, r))
        return set_error(TVS_E_UNSUPPORTED, "radius " + std::to_string(r) + " " +
                                                (shape == TVS_BOX ? "box" : "star") + " in " +
                                                std::to_string(ndim) +
                                                "D: every star and box of radius 2 and 3 but the "
                                                "3D radius-3 box (343 weights) is implemented");
    if (dependence == TVS_GAUSS_SEIDEL && boundary == TVS_PERIODIC)
        return set_error(TVS_E_UNSUPPORTED, "Gauss-Seidel with a periodic boundary");
    if (dependence == TVS_GAUSS_SEIDEL && ndim == 3 && dims[0] - 2 > 65535)
        return set_error(TVS_E_UNSUPPORTED, "3D Gauss-Seidel: axis 0 is limited to 65537 points");
    pr->ndim = ndim;
    for (int a = 0; a < 3; ++a) pr->dims[a] = a < ndim ? dims[a] : 1;
    pr->dtype = dtype;
    pr->shape = shape;
    pr->order = order;
    pr->dependence = dependence;
    pr->boundary = boundary;
    pr->radius = r;
    return TVS_OK;
}

// Game of Life B2S23 (Section 3.4, Table 1): a 2D 9-point box problem with
// Jacobi dependence on int32 cells.
int validate_life(Problem* pr, int ndim, const int64_t* dims, int boundary) {
    if (ndim != 2) return set_error(TVS_E_SHAPE, "Game of Life boards are 2D");
    int rc = validate(pr, ndim, dims, TVS_F32, TVS_BOX, 9, TVS_JACOBI, boundary);
    if (rc) return rc;
    pr->dtype = TVS_I32;
    pr->rule = TVS_RULE_LIFE;
    return TVS_OK;
}

// ---------------------------------------------------------------------------
// Tuning strings: "method=tstp,k=8,w=512,l=256,c=8,lanemap=1"
// ---------------------------------------------------------------------------
int parse_tuning(const char* str, Schedule* s, bool* has_method) {
    *has_method = false;
    if (!str) return TVS_OK;
    std::string t(str);
    size_t pos = 0;
    while (pos < t.size()) {
        size_t end = t.find(',', pos);
        if (end == std::string::npos) end = t.size();
        std::string kv = t.substr(pos, end - pos);
        pos = end + 1;
        if (kv.empty()) continue;
        size_t eq = kv.find('=');
        if (eq == std::string::npos) return set_error(TVS_E_INVALID, "tuning item without '=': " + kv);
        std::string key = kv.substr(0, eq), val = kv.substr(eq + 1);
        if (key == "method") {
            *has_method = true;
            if (val == "plain") s->method = TVS_METHOD_PLAIN;
            else if (val == "tstp") s->method = TVS_METHOD_TSTP;
            else return set_error(TVS_E_INVALID, "unknown method " + val);
            continue;
        }
        char* e = nullptr;
        long v = std::strtol(val.c_str(), &e, 10);
        if (!e || *e || val.empty() || v < 0 || v > (1 << 24))
            return set_error(TVS_E_INVALID, "bad tuning value " + kv);
        if (key == "k") s->k = (int)v;
        else if (key == "s") s->s = (int)v;
        else if (key == "w") s->w = (int)v;
        else if (key == "h") s->h = (int)v;
        else if (key == "l") s->l = (int)v;
        else if (key == "c") s->c = (int)v;
        else if (key == "lanemap") s->lanemap = (int)v;
        else if (key == "pl") s->pl = (int)v;
        else if (key == "kern") s->kern = (int)v;
        else return set_error(TVS_E_INVALID, "unknown tuning key " + key);
    }
    return TVS_OK;
}

std::string format_tuning(const Problem& p, const Schedule& s) {
    char buf[160];
    if (s.method == TVS_METHOD_PLAIN) return "method=plain";
    if (p.dependence == TVS_GAUSS_SEIDEL) {
        std::snprintf(buf, sizeof buf, "method=tstp,k=%d,c=%d", s.k, s.c);
    } else if (p.ndim == 1) {
        std::snprintf(buf, sizeof buf, "method=tstp,k=%d,l=%d,pl=%d", s.k, s.l, s.pl);
    } else {
        std::snprintf(buf, sizeof buf, "method=tstp,k=%d,w=%d,h=%d,l=%d,c=%d,lanemap=%d,kern=%d",
                      s.k, s.w, s.h, s.l, s.c, s.lanemap, s.kern);
    }
    return buf;
}

// Workgroups that fit on one CU for a band geometry (LDS and wave limits).
int wgs_per_cu(const BandGeom& g) {
    // the LDS pipelines use about 100-128 VGPRs (four waves per SIMD)
    int waves = std::max(1, (g.NT + 63) / 64);
    int by_waves = std::max(1, 16 / waves);
    int by_lds = g.lds_bytes ? (int)((160 * 1024) / g.lds_bytes) : by_waves;
    return std::max(1, std::min(by_waves, by_lds));
}

// Modelled time of one band, in units of "one step of one workgroup":
// rounds of the machine times steps per tile.
double band_cost(const Problem& p, const BandGeom& g) {
    const int cus = 256;
    const double slots = (double)cus * wgs_per_cu(g);
    const double tiles = (double)g.blocks();
    const double rounds = std::ceil(tiles / slots);
    const double steps = g.Lv + 3.0 * g.k * p.radius;
    return rounds * steps;
}

// Choose the stream-segment length for a geometry: the one with the least
// modelled time over all points, with full-machine rounds.  vc: the band
// kernel of variable coefficients (its LDS weight ring counted).
void choose_segment(const Problem& p, Schedule* s, bool vc) {
    if (p.ndim == 1) return;
    const int nstream = (int)p.dims[0];
    double best = 1e300;
    int best_l = s->l > 0 ? s->l : 256;
    for (int l = 32; l <= std::max(32, nstream); l += (l < 256 ? 8 : 16)) {
        Schedule t = *s;
        t.l = l;
        BandGeom g;
        if (vc ? !ndr_geometry(p, t, t.k, &g, true) : !band_geometry(p, t, t.k, &g)) continue;
        double c = band_cost(p, g);
        if (c < best - 1e-9) {
            best = c;
            best_l = l;
        }
        if (l >= nstream) break;
    }
    s->l = best_l;
}

Schedule default_schedule(const Problem& p) {
    Schedule s;
    s.method = TVS_METHOD_TSTP;
    if (p.dependence == TVS_GAUSS_SEIDEL) {
        // sweeps per launch.  1D: one lane per sweep, up to 16 waves (1024
        // sweeps) in one launch.  2D: more sweeps in flight hide the
        // dependency waits (measured best 128 on 4096^2, 64 on 600^2); one
        // row per lane.  3D: sweeps pipelined along the plane wavefront,
        // a group of k costs planes + G (k - 1) launches (measured best 64
        // on 800^3: 98.6 GStencil/s against 91.0 at 16 and 95.3 at 256).
        if (p.ndim == 1)
            s.k = 1024;
        else if (p.ndim == 2)
            s.k = p.dims[1] - 2 >= 2048 ? 128 : 64;
        else
            s.k = 64;
        s.c = 1;
        return s;
    }
    const bool f64 = p.dtype == TVS_F64;
    if (p.radius > 1 && p.ndim >= 2) {
        // the 2D/3D band kernel of radius r (skew 2r): R + 1 LDS rows per
        // level and 2r halo columns per level limit the depth
        s.s = 2 * p.radius;
        s.c = 4;
        s.lanemap = 1;
        if (p.ndim == 2) {
            s.k = 4;
            s.w = 256;
            while (s.w > 64 && s.w - 2 * s.k * p.radius > 2 * p.dims[1]) s.w /= 2;
        } else {
            s.k = 2;
            s.w = 32;
            s.h = 32;
            while (s.w > 16 && s.w - 2 * s.k * p.radius > 2 * p.dims[2]) s.w /= 2;
            while (s.h > 8 && s.h - 2 * s.k * p.radius > 2 * p.dims[1]) s.h /= 2;
        }
        while (s.k > 1 && (s.w <= 2 * s.k * p.radius || (p.ndim == 3 && s.h <= 2 * s.k * p.radius)))
            --s.k;
        choose_segment(p, &s);
        BandGeom g;
        if (!band_geometry(p, s, s.k, &g)) {
            Schedule plain;
            plain.method = TVS_METHOD_PLAIN;
            return plain;
        }
        return s;
    }
    if (p.radius > 1) {
        // radius > 1 in 1D: the 64-lane pipeline (skew r + 1)
        s.s = p.radius + 1;
        s.pl = 64;
        s.k = 64;
        s.l = 128;  // measured best on 1e5 points, radius 2 (64..512 tried)
        return s;
    }
    if (p.ndim == 1) {
        s.pl = 64;
        s.k = 64;
        int64_t n = p.dims[0];
        // short segments: many pipelines in flight (measured best 64 on
        // 1e5 points), longer ones on long grids
        int64_t l = (n + 2047) / 2048;
        s.l = (int)std::max<int64_t>(64, std::min<int64_t>(l, 4096));
        return s;
    }
    if (p.ndim == 2) {
        // measured best on 8192^2 box stencils (FP64 and FP32): 8 points per
        // lane, 8 levels, successive levels in successive waves
        s.c = 8;
        s.k = 8;
        s.w = 256;
        s.lanemap = 1;
        // narrow grids: shrink the tile so that it is not mostly halo
        while (s.w > 64 && s.w - 2 * s.k > 2 * p.dims[1]) s.w /= 2;
        if (s.w <= 2 * s.k) s.k = std::max(1, s.w / 4);
    } else {
        // measured best on 512^3 star stencils (FP64 and FP32): 4 levels on
        // 32 x 32 tiles, 8 points per lane
        s.c = 8;
        s.k = 4;
        s.w = 32;
        s.h = 32;
        s.lanemap = 0;
        (void)f64;
        while (s.w > 16 && s.w - 2 * s.k > 2 * p.dims[2]) s.w /= 2;
        while (s.h > 8 && s.h - 2 * s.k > 2 * p.dims[1]) s.h /= 2;
        while (s.w <= 2 * s.k || s.h <= 2 * s.k) --s.k;
        if (s.k < 1) s.k = 1;
        while (s.h * s.w / s.c * s.k > 512 && s.c < 16) s.c *= 2;
    }
    choose_segment(p, &s);
    // a grid the band kernels cannot take (e.g. a stream-axis plane of 2 GiB
    // or more) runs the plain sweep
    BandGeom g;
    if (!band_geometry(p, s, s.k, &g)) {
        Schedule plain;
        plain.method = TVS_METHOD_PLAIN;
        return plain;
    }
    return s;
}

// Is a schedule runnable for this problem (all bands it will need)?
// Schedule of variable-coefficient runs.  1D takes the plan's schedule.  2D
// and 3D run the band kernel with at most 4 points per lane; given: the
// plan's schedule came from a tuning string or the tuning cache (its tile
// and depth are kept), else a 2D radius-1 plan takes the geometry measured
// best with the LDS weight ring (4096^2 FP64 5-point: 8 levels on 128-wide
// tiles, 227 GStencil/s against 217 for 5 levels on 256 and 206 for 6 on
// 96).  The depth is lowered until the band fits the LDS.
Schedule varcoef_schedule(const Problem& p, const Schedule& s, bool given) {
    if (p.ndim == 1 || s.method != TVS_METHOD_TSTP) return s;
    Schedule v = s;
    v.c = std::min(v.c, 4);
    if (!given && p.ndim == 2 && p.radius == 1) {
        v.c = 4;
        v.k = 8;
        v.w = 128;
        v.lanemap = 1;
        // narrow grids: shrink the tile so that it is not mostly halo
        while (v.w > 32 && v.w - 2 * v.k > 2 * p.dims[1]) v.w /= 2;
        if (v.w <= 2 * v.k) v.k = std::max(1, v.w / 4);
        choose_segment(p, &v, true);
    }
    BandGeom g;
    while (v.k > 1 && !ndr_geometry(p, v, v.k, &g, true)) --v.k;
    return v;
}

int check_schedule(const Problem& p, const Schedule& s) {
    if (s.method == TVS_METHOD_PLAIN) return TVS_OK;
    if (s.k < 1) return set_error(TVS_E_INVALID, "k must be >= 1");
    if (s.kern != 0)
        return set_error(TVS_E_INVALID, "kern must be 0 (the LDS level-plane pipeline)");
    if (p.dependence == TVS_GAUSS_SEIDEL) {
        const int kmax = p.ndim == 2 ? 256 : 1024;
        if (s.k > kmax)
            return set_error(TVS_E_INVALID, "k must be <= " + std::to_string(kmax) +
                                                " for Gauss-Seidel in " + std::to_string(p.ndim) + "D");
        if (s.c != 1)
            return set_error(TVS_E_INVALID, "c (rows per lane) must be 1 for Gauss-Seidel");
        return TVS_OK;
    }
    if (p.radius > 1 && p.ndim >= 2) {
        if (s.s != 2 * p.radius)
            return set_error(TVS_E_INVALID, "skew s = 2r: the 2D/3D pipeline of radius r runs "
                                            "every level 2r stream rows behind the one below "
                                            "(legal: s > r)");
    } else if (p.radius > 1) {
        if (s.s != p.radius + 1)
            return set_error(TVS_E_INVALID, "skew s = r + 1 is the legal choice for radius r "
                                            "(s > max dx/dt)");
        if (s.pl != 64 || s.k > 64)
            return set_error(TVS_E_INVALID, "radius > 1: 64-lane pipelines (pl=64), k <= 64");
        if (tstp1d_radius_lds_bytes(p, s.k, s.l > 0 ? s.l : 256) > 160 * 1024)
            return set_error(TVS_E_INVALID, "segment too long for LDS: " + format_tuning(p, s));
    } else if (s.s != 2) {
        return set_error(TVS_E_INVALID, "skew s = 2 is the only legal choice for radius 1 "
                                        "(s > max dx/dt) with one barrier per step");
    }
    // the full band must fit; shallower remainder bands that do not fit the
    // tile shape run as plain steps
    BandGeom g;
    if (!band_geometry(p, s, s.k, &g))
        return set_error(TVS_E_INVALID, "schedule cannot run a band of " + std::to_string(s.k) +
                                            " levels: " + format_tuning(p, s));
    return TVS_OK;
}

}  // namespace tvs
