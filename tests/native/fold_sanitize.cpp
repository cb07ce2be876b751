// The kernels' streaming fold (fold_source in core.hpp) evaluated on the
// host for every node and velocity of many small grids, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host side by
// tests/test_native_sanitizers.py: every source must lie inside the grid and
// the pull must be a permutation of the populations (each source slot used
// exactly once).  Exits 0 on success.
#include <cstdio>
#include <vector>

#include "../../paper_1411_3133_amd/csrc/core.hpp"

using namespace mlbm;

int main()
{
    int grids = 0;
    for (int n1 : {4, 5, 7, 16})
        for (int n2 : {1, 3, 4})
            for (int n3 : {1, 4, 6, 13, 19})
                for (int walls : {0, 1, 4, 5, 9}) {
                    if ((walls & 4) && n3 < 4) continue;
                    InstDesc d{};
                    d.n1 = n1; d.n2 = n2; d.n3 = n3; d.walls = walls & 5;
                    d.eqwall = (walls & 8) ? 1 : 0;
                    d.P = n2 * n3; d.N = n1 * d.P; d.n3p = n3; d.Pp = d.P;
                    std::vector<int> used((size_t)Q * d.N, 0);
                    for (int x1 = 0; x1 < n1; ++x1)
                        for (int x2 = 0; x2 < n2; ++x2)
                            for (int x3 = 0; x3 < n3; ++x3) {
                                bool ok = true;
                                static_for<0, Q>([&](auto q) {
                                    bool flip = false;
                                    int row = 0;
                                    const int col = fold_source<CV[q][0], CV[q][1], CV[q][2]>(d, x1, x2, x3, flip, row);
                                    if (row < 0 || row >= n1 || col < 0 || col >= d.P) { ok = false; return; }
                                    const int qs = flip ? opposite(q) : (int)q;
                                    used[(size_t)((row * d.P + col)) * Q + qs] += 1;
                                });
                                if (!ok) {
                                    std::printf("source outside the grid: %d %d %d walls %d\n", n1, n2, n3, walls);
                                    return 1;
                                }
                            }
                    if (!d.eqwall)   // equilibrium walls read wall nodes several times: not a permutation
                        for (int u : used)
                            if (u != 1) {
                                std::printf("not a permutation: %d %d %d walls %d\n", n1, n2, n3, walls);
                                return 1;
                            }
                    ++grids;
                }
    std::printf("%d grids ok\n", grids);
    return 0;
}
