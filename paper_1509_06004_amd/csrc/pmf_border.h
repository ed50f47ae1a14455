// Arc directions of the grid and the layout of a tile's cross-tile inbox
// (shared by the device kernels and a host-side check of the layout).
#pragma once

#include "pmf_internal.h"

#if defined(__HIPCC__)
#define PMF_HD __host__ __device__
#else
#define PMF_HD
#endif

namespace pmf {

// Arc k leads from pixel (x, y) to (x + DXk(k), y + DYk(k)); k ^ 1 is the
// reverse arc.  4-connectivity uses k < 4.
PMF_HD constexpr int DXk(int k) {
    return k == 0 ? 1 : k == 1 ? -1 : k == 2 ? 0 : k == 3 ? 0 : k == 4 ? 1 : k == 5 ? -1 : k == 6 ? -1 : 1;
}
PMF_HD constexpr int DYk(int k) {
    return k == 0 ? 0 : k == 1 ? 0 : k == 2 ? 1 : k == 3 ? -1 : k == 4 ? 1 : k == 5 ? -1 : k == 6 ? 1 : -1;
}

// Inbox words of a tile: one per (border pixel, arc leaving the tile) pair,
// holding flow that the tile across the arc pushed into the pixel.  Words
// [0, AV*TW): the top row, arc a of the up-going arcs (3, 5, 7) at word
// a*TW + x; then the bottom row with the down-going arcs (2, 4, 6); then the
// left column with the left-going arcs (1, 5, 6) at a*TH + y; then the right
// column with (0, 4, 7).  A corner pixel's diagonal arc that leaves through
// the row is stored in the row, so its column word is never written.
template <int K, int TW, int TH>
struct Border {
    static constexpr int AV = K == 4 ? 1 : 3;  // arcs leaving through one row
    static constexpr int AH = K == 4 ? 1 : 3;  // arcs leaving through one column
    static constexpr int E = 2 * AV * TW + 2 * AH * TH;
    static_assert(E == border_words(K, TW, TH), "inbox size agrees with the host");
    // word of arc k at tile pixel (bx, by); the arc must leave the tile
    PMF_HD static inline int index(int bx, int by, int k) {
        const int dx = DXk(k), dy = DYk(k);
        const int ah = k < 2 ? 0 : (k == 4 || k == 5) ? 1 : 2;
        if (dy < 0 && by == 0) return ((k - 3) >> 1) * TW + bx;
        if (dy > 0 && by == TH - 1) return AV * TW + ((k - 2) >> 1) * TW + bx;
        if (dx < 0) return 2 * AV * TW + ah * TH + by;
        return 2 * AV * TW + AH * TH + ah * TH + by;
    }
    // the pair of word i (0 <= i < E)
    PMF_HD static inline void pair(int i, int &bx, int &by, int &k) {
        if (i < 2 * AV * TW) {
            const int bot = i >= AV * TW;
            const int j = i - bot * AV * TW, a = j / TW;
            bx = j - a * TW;
            by = bot ? TH - 1 : 0;
            k = (bot ? 2 : 3) + 2 * a;
        } else {
            const int j0 = i - 2 * AV * TW;
            const int rgt = j0 >= AH * TH;
            const int j = j0 - rgt * AH * TH, a = j / TH;
            by = j - a * TH;
            bx = rgt ? TW - 1 : 0;
            k = rgt ? (a == 0 ? 0 : a == 1 ? 4 : 7) : (a == 0 ? 1 : a == 1 ? 5 : 6);
        }
    }
};

}  // namespace pmf
