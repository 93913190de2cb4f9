// Host check of the population layout of csrc/lattice.h: for a lattice of
// pitch x ny nodes, element 64 i + tix<T>(k) of a state (array i's pointer
// is the state's base plus 64 i values when the layout is tiled, else
// array i is a separate range) must be distinct for every (array i, node k)
// and lie inside the 14 pitch ny values of the state.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lattice.h"

using namespace ptlbm;

template <class T>
static int check(size_t pitch, size_t ny) {
    const size_t n = pitch * ny, total = 14 * n;
    std::vector<unsigned char> seen(total, 0);
    for (int i = 0; i < 14; ++i)
        for (size_t k = 0; k < n; ++k) {
            const size_t e = tiled<T>() ? 64 * (size_t)i + tix<T>(k) : (size_t)i * n + tix<T>(k);
            if (e >= total) {
                std::printf("out of range: pitch %zu ny %zu array %d node %zu element %zu\n", pitch, ny, i, k, e);
                return 1;
            }
            if (seen[e]++) {
                std::printf("shared element: pitch %zu ny %zu array %d node %zu element %zu\n", pitch, ny, i, k, e);
                return 1;
            }
        }
    return 0;
}

int main() {
    const size_t shapes[][2] = {{64, 1}, {64, 9}, {128, 3}, {320, 70}, {4032, 4000}, {65536, 2}};
    for (const auto& sh : shapes) {
        if (check<double>(sh[0], sh[1]) || check<float>(sh[0], sh[1]) || check<unsigned short>(sh[0], sh[1]))
            return 1;
    }
    std::printf("layout ok\n");
    return 0;
}
