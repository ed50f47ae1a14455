// Kernels of the breakpoint searches (pmf_parametric, pmf_breakpoints): set
// statistics and exit maps of the integer search; for the real-lambda search,
// graph contraction of the pixels that leave the minimal source set inside
// one unit lambda interval, scaling of a contracted problem to a rational
// lambda, and the per-pixel exit bookkeeping.
#pragma once

#include <stdint.h>

namespace pmf {

// out[0] += |S|, out[1] += sum of the sink slopes of the free pixels in S, for
// a row-major mask of n pixels (out zeroed by the caller).
int launch_mask_stats(const uint8_t *mask, int n, const int32_t *slope, const uint8_t *seed, int64_t *out,
                      void *stream);

// out[p] = min(out[p], lam) where mask[p] == 0 (n pixels); out[p] = v.
int launch_exit_min(const uint8_t *mask, int n, int32_t lam, int32_t *out, void *stream);
int launch_fill_i32(int32_t *out, int n, int32_t v, void *stream);

// Per-interval statistics written by launch_contract (int64 each).
enum ContractStat : int {
    kCsD = 0,    // pixels of D
    kCsSumCs,    // sum over D of the contracted source capacity
    kCsSumC0,    // sum over D of the contracted sink capacity at lambda 0
    kCsSumSl,    // sum over D of the sink slope
    kCsMaxCs,    // largest contracted source capacity in D
    kCsMaxC0,    // largest contracted sink capacity at lambda 0 in D
    kCsMaxNl,    // largest n-link between two pixels of D
    kCsMaxSl,    // largest sink slope in D
    kCsSeeds,    // seed pixels in D (0 unless capacities reach INF)
    kCsCount
};

// boxes[4 i .. 4 i + 3] = {x_min, y_min, x_max, y_max} of the pixels p with
// exit[p] == changes[i] (changes: k ascending values; W x H exit map).
int launch_change_boxes(const int32_t *exit, int W, int H, const int32_t *changes, int k, int32_t *boxes,
                        void *stream);

// Contract the problem (nlink, cap_src, cap_snk0, slope, seed: a W x H
// instance with K-connectivity) to D = {p : exit[p] == c}, cropped to the box
// (x0, y0, w, h) that holds D.  With S1 = {exit >= c} and S2 = {exit > c}
// the pixels of S2 are merged into the source and those outside S1 into the
// sink: a pixel of D gets source capacity cs + the n-links into it from S2
// and sink capacity at lambda 0 c0 + its n-links into pixels outside S1; the
// n-links between pixels of D stay, every other capacity of the box is 0.
// planes: int32 [K + 3][h][w] = n-links (K planes), cs, c0, slope; ep / eq:
// int32 [h][w] exit value c / 1 on D, -1 / 1 elsewhere; stats: int64
// [kCsCount], zeroed here before the kernel adds to it.
int launch_contract(const int32_t *nlink, const int32_t *cap_src, const int32_t *cap_snk0, const int32_t *slope,
                    const uint8_t *seed, int W, int H, int K, const int32_t *exit, int32_t c, int x0, int y0, int w,
                    int h, int32_t *planes, int32_t *ep, int32_t *eq, int64_t *stats, void *stream);

// out[i] = in[i] * q for count int32 values (the caller has checked that no
// product leaves int32).
int launch_scale(const int32_t *in, int64_t count, int32_t q, int32_t *out, void *stream);

// For each of the n pixels with ep >= 0 that `mask` does not hold: ep / eq =
// min(ep / eq, p / q) (exact: cross-multiplied in int64).
int launch_exit_rational(const uint8_t *mask, int n, int32_t p, int32_t q, int32_t *ep, int32_t *eq,
                         void *stream);

// exit[p] (n pixels): lo -> 0, hi + 1 -> last, any other value -> -1.
int launch_exit_pieces_init(int32_t *exit, int n, int32_t lo, int32_t hi, int32_t last, void *stream);

// For each pixel of the box with ep >= 0: the index j of ep / eq among the nb
// ascending fractions bp (int64 pairs num, den), and exit[y * W + x] =
// base + j + 1 (-2 if absent).
int launch_exit_place(const int32_t *ep, const int32_t *eq, int x0, int y0, int w, int h, int W, const int64_t *bp,
                      int nb, int32_t base, int32_t *exit, void *stream);

}  // namespace pmf
