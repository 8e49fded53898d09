// Host-only listing of the 2D Gauss-Seidel item order (gs_order.hpp): for
// each case "nb sweeps", the order as "all: b,t b,t ...".  The test compares
// it with a brute-force enumeration and replays the kernel's waits on it.
#include <cstdio>

#include "../paper_2010_04868_amd/csrc/gs_order.hpp"

using namespace tvs::gs;

int main() {
    const int cases[][2] = {{1, 1}, {1, 5}, {3, 4}, {8, 1}, {9, 3}, {16, 7}, {17, 2},
                            {40, 9}, {64, 100}, {65, 33}};
    for (const auto& c : cases) {
        const int nb = c[0], sweeps = c[1];
        std::printf("case %d %d\n", nb, sweeps);
        std::printf("all:");
        for (int i = 0; i < nb * sweeps; ++i) {
            int b, t;
            decode_item(i, nb, sweeps, &b, &t);
            std::printf(" %d,%d", b, t);
        }
        std::printf("\n");
    }
    return 0;
}
