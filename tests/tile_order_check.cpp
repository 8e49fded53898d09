// Host-only check of the band kernel's tile dispatch order: for many grids,
// tile shapes and depths, tile_order (with the interior ranges make_args
// computes) must be a bijection on the band's tiles and must list every tile
// that touches a fixed border before every interior tile.
#include <cstdio>
#include <vector>

#include "../paper_2010_04868_amd/csrc/tstp_nd.hpp"

using namespace tvs;

int main() {
    long cases = 0, bad = 0;
    for (int D = 2; D <= 3; ++D)
        for (int per = 0; per <= 1; ++per)
            for (int nz : {5, 17, 300, 1000})
                for (int ny : {5, 33, 200})
                    for (int nx : {5, 40, 129, 700})
                        for (int k : {1, 2, 3, 8})
                            for (int w : {16, 64, 256})
                                for (int h : {8, 32})
                                    for (int l : {16, 96, 288}) {
                                        if (D == 2 && (ny != 5 || h != 8)) continue;
                                        Problem p;
                                        p.ndim = D;
                                        p.dtype = TVS_F64;
                                        p.shape = TVS_STAR;
                                        p.order = 2 * D + 1;
                                        p.boundary = per ? TVS_PERIODIC : TVS_DIRICHLET;
                                        p.dims[0] = nz;
                                        p.dims[1] = D == 3 ? ny : nx;
                                        p.dims[2] = D == 3 ? nx : 1;
                                        Schedule s;
                                        s.method = TVS_METHOD_TSTP;
                                        s.k = k;
                                        s.w = w;
                                        s.h = h;
                                        s.l = l;
                                        s.c = 4;
                                        BandGeom g;
                                        if (!band_geometry(p, s, k, &g)) continue;
                                        const nd::ArgsNd a = nd::make_args(p, g);
                                        const int tiles = a.ntx * a.nty * a.nseg;
                                        auto border = [&](int t) {
                                            const int bx = t % a.ntx, by = (t / a.ntx) % a.nty,
                                                      bs = t / (a.ntx * a.nty);
                                            const int xo = bx * a.Wv - k, yo = by * a.Hv - k,
                                                      zo = bs * a.Lv - k;
                                            bool b = xo <= 0 || xo + a.W - 1 >= a.nx - 1 ||
                                                     zo <= 0 || zo + a.Lin - 1 >= a.nz - 1;
                                            if (D == 3) b = b || yo <= 0 || yo + a.H - 1 >= a.ny - 1;
                                            return !per && b;
                                        };
                                        std::vector<int> seen(tiles, 0);
                                        bool ok = true, border_phase = true;
                                        for (int blk = 0; blk < tiles && ok; ++blk) {
                                            const int t = nd::tile_order(blk, a);
                                            if (t < 0 || t >= tiles || seen[t]++) ok = false;
                                            else if (border(t) && !border_phase) ok = false;
                                            else if (!border(t)) border_phase = false;
                                        }
                                        ++cases;
                                        if (!ok && bad++ < 5)
                                            std::printf("FAIL D=%d per=%d dims=%d,%d,%d k=%d w=%d h=%d l=%d\n",
                                                        D, per, nz, ny, nx, k, w, h, l);
                                    }
    std::printf("%ld cases, %ld failures\n", cases, bad);
    return bad != 0 || cases < 1000;
}
