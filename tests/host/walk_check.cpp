// The work walks of the persistent pass kernels (fsa_walk.hpp), run for every
// workgroup of a grid on the CPU: each mode must visit every item exactly
// once, in increasing order per workgroup (the job-table cursor relies on
// it), for grids of 1 ... 2048 workgroups and item counts from the grid size
// up (a persistent grid never exceeds its items).  The pair walk must also
// give the two tiles of a pair to workgroups g and g + 8 (one XCD) wherever
// it applies.  Exit status 0 = pass.
#include <cstdio>
#include <vector>

#include "../../paper_2504_19410_amd/csrc/fsa_walk.hpp"

using namespace fsa;

template <int MODE>
static bool check(int items, int G) {
    std::vector<int> seen(items, 0), owner(items, -1);
    for (int g = 0; g < G; ++g) {
        const Walk w = Walk::make<MODE>(items, G, g);
        if (w.stride < 1) return false;
        int prev = -1;
        for (int it = w.first; it < w.last; it += w.stride) {
            if (it < 0 || it >= items || it <= prev) {
                std::printf("mode %d items %d G %d g %d: item %d out of range or order\n", MODE,
                            items, G, g, it);
                return false;
            }
            prev = it;
            ++seen[it];
            owner[it] = g;
        }
    }
    for (int i = 0; i < items; ++i)
        if (seen[i] != 1) {
            std::printf("mode %d items %d G %d: item %d visited %d times\n", MODE, items, G, i,
                        seen[i]);
            return false;
        }
    if (MODE == kWalkPair && G >= 16 && G % 16 == 0)
        for (int i = 0; i + 1 < items; i += 2)
            if (owner[i + 1] != owner[i] + 8) {
                std::printf("pair walk items %d G %d: tiles %d, %d on workgroups %d, %d\n", items,
                            G, i, i + 1, owner[i], owner[i + 1]);
                return false;
            }
    return true;
}

int main() {
    long cases = 0;
    for (int G = 1; G <= 2048; G = G < 64 ? G + 1 : G + 16)
        for (int items = G; items <= 40000; items += items < 700 ? 1 : 211) {
            if (!check<kWalkChunk>(items, G) || !check<kWalkXcd>(items, G) ||
                !check<kWalkPair>(items, G))
                return 1;
            ++cases;
        }
    std::printf("OK %ld grid / item-count cases, three modes\n", cases);
    return 0;
}
