// D3Q41 lattice of Table I (Sec. II) for the gfx950 kernels.
//
// The velocity order is that of Table I (rest, then the +-1 axis pairs, the
// (+-1,+-1,0)-type, (+-1,+-1,+-1), (+-3,0,0)-type and (+-3,+-3,+-3) groups,
// "+" first and the last component fastest inside a group).  The kernels
// work on the 20 (c, -c) pairs; every pair is a multiple k in {1, 3} of one
// of 13 unit directions, so the +-3 pairs reuse the direction quantities of
// the +-1 pairs (c = k * chat).
#pragma once

namespace mlbm {

constexpr int Q = 41;
constexpr int NPAIR = 20;
constexpr int NDIR = 13;

constexpr double SQRT10 = 3.16227766016837933199889354443271853;
// c_s^2 = 1 - sqrt(2/5)
constexpr double CS2 = 1.0 - 0.632455532033675866399778708886543707;

// Table I weight classes
constexpr double W_REST = 2.0 / 2025.0 * (5045.0 - 1507.0 * SQRT10);
constexpr double W_AX1 = 37.0 / (5.0 * SQRT10) - 91.0 / 40.0;
constexpr double W_PL1 = (55.0 - 17.0 * SQRT10) / 50.0;
constexpr double W_DI1 = (233.0 * SQRT10 - 730.0) / 1600.0;
constexpr double W_AX3 = (295.0 - 92.0 * SQRT10) / 16200.0;
constexpr double W_DI3 = (130.0 - 41.0 * SQRT10) / 129600.0;

// velocity table in Table I order
constexpr int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0},
    {1, 0, 1}, {1, 0, -1}, {-1, 0, 1}, {-1, 0, -1},
    {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1},
    {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1},
    {-1, 1, 1}, {-1, 1, -1}, {-1, -1, 1}, {-1, -1, -1},
    {3, 0, 0}, {-3, 0, 0}, {0, 3, 0}, {0, -3, 0}, {0, 0, 3}, {0, 0, -3},
    {3, 3, 3}, {3, 3, -3}, {3, -3, 3}, {3, -3, -3},
    {-3, 3, 3}, {-3, 3, -3}, {-3, -3, 3}, {-3, -3, -3},
};

constexpr double wq(int q)
{
    return q == 0 ? W_REST : q <= 6 ? W_AX1 : q <= 18 ? W_PL1 : q <= 26 ? W_DI1 : q <= 32 ? W_AX3 : W_DI3;
}

// unit directions chat (the "+" member of each pair, divided by k)
constexpr int DIR[NDIR][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1},
    {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1},
};

// (direction, k, q of +k chat, q of -k chat)
constexpr int PAIR[NPAIR][4] = {
    {0, 1, 1, 2}, {1, 1, 3, 4}, {2, 1, 5, 6},
    {3, 1, 7, 10}, {4, 1, 8, 9}, {5, 1, 11, 14}, {6, 1, 12, 13}, {7, 1, 15, 18}, {8, 1, 16, 17},
    {9, 1, 19, 26}, {10, 1, 20, 25}, {11, 1, 21, 24}, {12, 1, 22, 23},
    {0, 3, 27, 28}, {1, 3, 29, 30}, {2, 3, 31, 32},
    {9, 3, 33, 40}, {10, 3, 34, 39}, {11, 3, 35, 38}, {12, 3, 36, 37},
};

constexpr int opposite(int q)
{
    for (int p = 0; p < Q; ++p)
        if (CV[p][0] == -CV[q][0] && CV[p][1] == -CV[q][1] && CV[p][2] == -CV[q][2]) return p;
    return -1;
}

constexpr int cmax(int q)
{
    int m = 0;
    for (int a = 0; a < 3; ++a) {
        int v = CV[q][a] < 0 ? -CV[q][a] : CV[q][a];
        if (v > m) m = v;
    }
    return m;
}

}  // namespace mlbm
