// Kernels of the breakpoint searches: the size and slope sum of a minimal
// source set and the running exit map of the integer search, and for the
// exact real-lambda search the contraction of one unit lambda interval's
// changing pixels (Sec. 2.1: the minimal source sets are nested in lambda, so
// between two nested sets the outer pixels are fixed to the sink and the
// inner ones to the source, as in the parametric algorithm of Gallo,
// Grigoriadis and Tarjan), scaling to a rational lambda, and the per-pixel
// exit bookkeeping.  All are one pass over a mask or a box, bound by memory
// latency; the reductions combine a wave's lanes by shuffles before any
// atomic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "pmf.h"
#include "pmf_border.h"
#include "pmf_parametric.h"

namespace pmf {

namespace {

constexpr int kBlock = 256;

inline int blocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_fill_boxes(int32_t *boxes, int k) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < k) {
        boxes[4 * i] = INT_MAX;
        boxes[4 * i + 1] = INT_MAX;
        boxes[4 * i + 2] = -1;
        boxes[4 * i + 3] = -1;
    }
}

// A wave's lanes that hold pixels of the same change point combine their
// boxes by shuffles first (neighbouring pixels mostly leave together), so a
// change point of many pixels costs one set of atomics per wave, not per pixel.
__global__ __launch_bounds__(kBlock) void k_change_boxes(const int32_t *exit, int W, int n, const int32_t *changes,
                                                         int k, int32_t *boxes) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    int idx = -1;
    if (p < n) {
        const int32_t e = exit[p];
        int lo = 0, hi = k;  // first change >= e
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (changes[mid] < e)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo < k && changes[lo] == e) idx = lo;
    }
    const int x = p % W, y = p / W, lane = (int)(threadIdx.x & 63);
    unsigned long long left = __ballot(idx >= 0);
    while (left) {  // wave-uniform
        const int leader = __ffsll((long long)left) - 1;
        const int li = __shfl(idx, leader);
        const bool mine = idx == li;
        int x0 = mine ? x : INT_MAX, y0 = mine ? y : INT_MAX, x1 = mine ? x : -1, y1 = mine ? y : -1;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            x0 = min(x0, __shfl_xor(x0, off));
            y0 = min(y0, __shfl_xor(y0, off));
            x1 = max(x1, __shfl_xor(x1, off));
            y1 = max(y1, __shfl_xor(y1, off));
        }
        if (lane == leader) {
            atomicMin(&boxes[4 * li], x0);
            atomicMin(&boxes[4 * li + 1], y0);
            atomicMax(&boxes[4 * li + 2], x1);
            atomicMax(&boxes[4 * li + 3], y1);
        }
        left &= ~__ballot(mine);
    }
}

// Size and slope sum of a mask: a grid-stride pass, the lanes' sums combined
// by shuffles, then the waves' in LDS, one pair of atomics per workgroup.
__global__ __launch_bounds__(kBlock) void k_mask_stats(const uint8_t *mask, int n, const int32_t *slope,
                                                       const uint8_t *seed, unsigned long long *out) {
    __shared__ long long s_in[kBlock / 64], s_w[kBlock / 64];
    long long in = 0, w = 0;
    for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) {
        if (mask[p]) {
            in += 1;
            if (!seed || seed[p] == 0) w += slope ? slope[p] : 1;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        in += __shfl_xor(in, off);
        w += __shfl_xor(w, off);
    }
    const int wv = (int)(threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0) {
        s_in[wv] = in;
        s_w[wv] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long ti = 0, tw = 0;
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) {
            ti += s_in[i];
            tw += s_w[i];
        }
        if (ti) atomicAdd(&out[0], (unsigned long long)ti);
        if (tw) atomicAdd(&out[1], (unsigned long long)tw);
    }
}

// out[p] = min(out[p], lam) for every pixel p that `mask` (n bytes) does not
// hold.  Applied to the masks of several lambdas it leaves, per pixel, the
// smallest of those lambdas whose minimal source set lacks the pixel.
__global__ __launch_bounds__(kBlock) void k_exit_min(const uint8_t *mask, int n, int32_t lam, int32_t *out) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < n && !mask[p] && lam < out[p]) out[p] = lam;
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *out, int n, int32_t v) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < n) out[p] = v;
}

__global__ __launch_bounds__(kBlock) void k_zero_i64(int64_t *out, int n) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_contract(const int32_t *nlink, const int32_t *cap_src,
                                                     const int32_t *cap_snk0, const int32_t *slope,
                                                     const uint8_t *seed, int W, int H, int K, const int32_t *exit,
                                                     int32_t c, int x0, int y0, int w, int h, int32_t *planes,
                                                     int32_t *ep, int32_t *eq, unsigned long long *stats) {
    __shared__ unsigned long long s[kCsCount];
    if (threadIdx.x < kCsCount) s[threadIdx.x] = 0;
    __syncthreads();
    const int a = w * h;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < a) {
        const int x = x0 + i % w, y = y0 + i / w;
        const size_t n = (size_t)W * H, gp = (size_t)y * W + x;
        const bool in_d = exit[gp] == c;
        int64_t cs = 0, c0 = 0, sl = 0, mx_nl = 0;
        for (int k = 0; k < K; ++k) {
            int32_t v = 0;
            if (in_d) {
                // the arc p -> q (q = p + d_k): kept inside D, moved to the
                // sink capacity when q is outside S1, gone when q is in S2
                const int qx = x + DXk(k), qy = y + DYk(k);
                if (qx >= 0 && qy >= 0 && qx < W && qy < H) {
                    const int32_t eq_ = exit[(size_t)qy * W + qx];
                    const int32_t cap = nlink[(size_t)k * n + gp];
                    if (eq_ == c) {
                        v = cap;
                        mx_nl = cap > mx_nl ? cap : mx_nl;
                    } else if (eq_ < c) {
                        c0 += cap;
                    }
                }
                // the arc u -> p (u = p - d_k): moved to the source capacity
                // when u is in S2
                const int ux = x - DXk(k), uy = y - DYk(k);
                if (ux >= 0 && uy >= 0 && ux < W && uy < H) {
                    const size_t u = (size_t)uy * W + ux;
                    if (exit[u] > c) cs += nlink[(size_t)k * n + u];
                }
            }
            planes[(size_t)k * a + i] = v;
        }
        int32_t *pcs = planes + (size_t)K * a, *pc0 = pcs + a, *psl = pc0 + a;
        if (in_d) {
            cs += cap_src[gp];
            c0 += cap_snk0[gp];
            sl = slope ? slope[gp] : 1;
            const bool is_seed = seed && seed[gp] != 0;
            // sums stay far below 2^63; values above int32 are refused by the
            // caller from the maxima before any product is formed
            pcs[i] = cs > INT_MAX ? INT_MAX : (int32_t)cs;
            pc0[i] = c0 > INT_MAX ? INT_MAX : (int32_t)c0;
            psl[i] = (int32_t)sl;
            ep[i] = c;
            atomicAdd(&s[kCsD], 1ull);
            atomicAdd(&s[kCsSumCs], (unsigned long long)cs);
            atomicAdd(&s[kCsSumC0], (unsigned long long)c0);
            atomicAdd(&s[kCsSumSl], (unsigned long long)sl);
            atomicMax(&s[kCsMaxCs], (unsigned long long)cs);
            atomicMax(&s[kCsMaxC0], (unsigned long long)c0);
            atomicMax(&s[kCsMaxNl], (unsigned long long)mx_nl);
            atomicMax(&s[kCsMaxSl], (unsigned long long)sl);
            if (is_seed) atomicAdd(&s[kCsSeeds], 1ull);
        } else {
            pcs[i] = 0;
            pc0[i] = 0;
            psl[i] = 0;
            ep[i] = -1;
        }
        eq[i] = 1;
    }
    __syncthreads();
    if (threadIdx.x < kCsCount && s[threadIdx.x]) {
        const int t = threadIdx.x;
        if (t >= kCsMaxCs && t <= kCsMaxSl)
            atomicMax(&stats[t], s[t]);
        else
            atomicAdd(&stats[t], s[t]);
    }
}

__global__ __launch_bounds__(kBlock) void k_scale(const int32_t *in, int64_t count, int32_t q, int32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) out[i] = (int32_t)((int64_t)in[i] * q);
}

__global__ __launch_bounds__(kBlock) void k_exit_rational(const uint8_t *mask, int n, int32_t p, int32_t q,
                                                          int32_t *ep, int32_t *eq) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || mask[i]) return;
    const int32_t e = ep[i];
    if (e < 0) return;
    if ((int64_t)p * eq[i] < (int64_t)e * q) {
        ep[i] = p;
        eq[i] = q;
    }
}

__global__ __launch_bounds__(kBlock) void k_exit_pieces_init(int32_t *exit, int n, int32_t lo, int32_t hi,
                                                             int32_t last) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t v = exit[i];
    exit[i] = v == lo ? 0 : (int64_t)v == (int64_t)hi + 1 ? last : -1;
}

__global__ __launch_bounds__(kBlock) void k_exit_place(const int32_t *ep, const int32_t *eq, int x0, int y0, int w,
                                                       int h, int W, const int64_t *bp, int nb, int32_t base,
                                                       int32_t *exit) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= w * h || ep[i] < 0) return;
    const int64_t p = ep[i], q = eq[i];
    int lo = 0, hi = nb;  // first breakpoint >= p / q
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (bp[2 * mid] * q < p * bp[2 * mid + 1])
            lo = mid + 1;
        else
            hi = mid;
    }
    const bool hit = lo < nb && bp[2 * lo] * q == p * bp[2 * lo + 1];
    exit[(size_t)(y0 + i / w) * W + x0 + i % w] = hit ? base + lo + 1 : -2;
}

inline int launched() { return hipGetLastError() == hipSuccess ? 0 : -1; }

}  // namespace

int launch_mask_stats(const uint8_t *mask, int n, const int32_t *slope, const uint8_t *seed, int64_t *out,
                      void *stream) {
    hipLaunchKernelGGL(k_mask_stats, dim3(std::min(blocks(n), 256)), dim3(kBlock), 0, (hipStream_t)stream, mask, n,
                       slope, seed, (unsigned long long *)out);
    return launched();
}

int launch_exit_min(const uint8_t *mask, int n, int32_t lam, int32_t *out, void *stream) {
    hipLaunchKernelGGL(k_exit_min, dim3(blocks(n)), dim3(kBlock), 0, (hipStream_t)stream, mask, n, lam, out);
    return launched();
}

int launch_fill_i32(int32_t *out, int n, int32_t v, void *stream) {
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(n)), dim3(kBlock), 0, (hipStream_t)stream, out, n, v);
    return launched();
}

int launch_change_boxes(const int32_t *exit, int W, int H, const int32_t *changes, int k, int32_t *boxes,
                        void *stream) {
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill_boxes, dim3(blocks(k)), dim3(kBlock), 0, s, boxes, k);
    hipLaunchKernelGGL(k_change_boxes, dim3(blocks((int64_t)W * H)), dim3(kBlock), 0, s, exit, W, W * H, changes, k,
                       boxes);
    return launched();
}

int launch_contract(const int32_t *nlink, const int32_t *cap_src, const int32_t *cap_snk0, const int32_t *slope,
                    const uint8_t *seed, int W, int H, int K, const int32_t *exit, int32_t c, int x0, int y0, int w,
                    int h, int32_t *planes, int32_t *ep, int32_t *eq, int64_t *stats, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(kBlock), 0, s, stats, (int)kCsCount);
    hipLaunchKernelGGL(k_contract, dim3(blocks((int64_t)w * h)), dim3(kBlock), 0, s, nlink, cap_src, cap_snk0, slope,
                       seed, W, H, K, exit, c, x0, y0, w, h, planes, ep, eq, (unsigned long long *)stats);
    return launched();
}

int launch_scale(const int32_t *in, int64_t count, int32_t q, int32_t *out, void *stream) {
    hipLaunchKernelGGL(k_scale, dim3(blocks(count)), dim3(kBlock), 0, (hipStream_t)stream, in, count, q, out);
    return launched();
}

int launch_exit_rational(const uint8_t *mask, int n, int32_t p, int32_t q, int32_t *ep, int32_t *eq,
                         void *stream) {
    hipLaunchKernelGGL(k_exit_rational, dim3(blocks(n)), dim3(kBlock), 0, (hipStream_t)stream, mask, n, p, q, ep,
                       eq);
    return launched();
}

int launch_exit_pieces_init(int32_t *exit, int n, int32_t lo, int32_t hi, int32_t last, void *stream) {
    hipLaunchKernelGGL(k_exit_pieces_init, dim3(blocks(n)), dim3(kBlock), 0, (hipStream_t)stream, exit, n, lo, hi,
                       last);
    return launched();
}

int launch_exit_place(const int32_t *ep, const int32_t *eq, int x0, int y0, int w, int h, int W, const int64_t *bp,
                      int nb, int32_t base, int32_t *exit, void *stream) {
    hipLaunchKernelGGL(k_exit_place, dim3(blocks((int64_t)w * h)), dim3(kBlock), 0, (hipStream_t)stream, ep, eq, x0,
                       y0, w, h, W, bp, nb, base, exit);
    return launched();
}

}  // namespace pmf
