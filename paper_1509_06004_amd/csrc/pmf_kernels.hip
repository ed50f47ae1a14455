// HIP kernels of libpmf for gfx950: exact push-relabel max-flow on grid graphs.
//
// Method (paper Sec. 2: s-t graph of an image, max flow = min cut; Sec. 2.1:
// monotone parametric capacities solved over a lambda schedule, nested
// optimal cuts; Sec. 3.1: many graphs solved together as one "supergraph").
// The push-relabel algorithm the paper runs as a closed library is rebuilt
// here from its textbook definition (Goldberg-Tarjan), with exact global
// relabelling by breadth-first search (Cherkassky-Goldberg):
//
//   - a *superstep* is three launches: a compaction kernel lists the tiles
//     that have work, a tile kernel processes them (each workgroup takes one
//     TW x TH tile of one instance at a time and performs that instance's
//     current phase on it), and a control kernel advances every instance's
//     phase machine; supersteps are replayed from a captured graph with no
//     host round trip in between;
//   - kSweep: the tile's state is loaded into registers / LDS and up to
//     `inner_iters` push/relabel iterations run against halo heights; pushes
//     that leave the tile are accumulated and handed to the neighbour tile
//     through its atomic inbox;
//   - kRelabel: exact distances to t by tile-parallel Bellman-Ford relaxation
//     (tile-local relaxation to a fixed point, repeated over the tiles whose
//     neighbourhood changed).  A pass in which no label changes proves the
//     distances exact; pixels that cannot reach t get H_INF (at that instant
//     every vertex above an empty level is among them; between relabels the
//     optional gap heuristic finds levels that the sweeps empty).  If no
//     pixel with excess can still reach t, the preflow is maximum;
//   - kCut: the minimal source side is the set of pixels reachable in the
//     residual graph from the pixels still holding excess (all source arcs
//     stay saturated, so s itself reaches nothing else);
//   - F = (total source capacity) - (total excess left on pixels);
//   - warm start: after a lambda is finished the sink residuals grow by
//     slope * (lambda' - lambda); the preflow stays feasible, so the next
//     lambda continues from it after a fresh global relabel.
//
// Correctness never depends on labels being valid between global relabels:
// the bookkeeping is exact integer arithmetic and termination is certified by
// an exact relabel on a quiescent state.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pmf.h"
#include "pmf_border.h"
#include "pmf_internal.h"

namespace pmf {


template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Instance arrays live in device global memory.  Their pointers are read from
// the descriptor table, so the compiler cannot tell their address space and
// would emit flat instructions (which count against the LDS wait counter as
// well); gp() states it, giving global loads, stores and atomics.
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T *gp(T *p) {
    return (GLOBAL T *)p;
}
// Descriptors are written by the host before any launch and only read by the
// kernels: a workgroup-uniform descriptor read goes through the constant
// address space, i.e. scalar loads.
__device__ __forceinline__ InstDesc load_desc(const InstDesc *table, int slot) {
    static_assert(sizeof(InstDesc) % 4 == 0, "descriptor read in 4-byte words");
    const __attribute__((address_space(4))) uint32_t *src =
        (const __attribute__((address_space(4))) uint32_t *)(table + slot);
    InstDesc d;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&d);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(InstDesc) / 4); ++i) dst[i] = src[i];
    return d;
}
template <typename T>
__device__ __forceinline__ T ld_agent(GLOBAL const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(GLOBAL T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void g_add(GLOBAL T *p, T v) {
    (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void g_or(GLOBAL T *p, T v) {
    (void)__hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void g_and(GLOBAL T *p, T v) {
    (void)__hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int TW, int TH>
struct Geo {
    static constexpr int NT = kThreads;
    static constexpr int PPT = TW * TH / NT;  // pixels per thread
    static constexpr int RPI = NT / TW;       // rows covered by one pass of the block
    static constexpr int HW = TW + 2;
    static constexpr int HH = TH + 2;
    static constexpr int HALO = HW * HH;
    static constexpr int RING = 2 * HW + 2 * TH;
    static_assert(TW * TH % NT == 0, "tile must be a multiple of the block");
    static_assert(NT % TW == 0, "tile width must divide the block");
    __device__ static inline void ring(int i, int &hx, int &hy) {
        if (i < HW) {
            hx = i;
            hy = 0;
        } else if (i < 2 * HW) {
            hx = i - HW;
            hy = HH - 1;
        } else if (i < 2 * HW + TH) {
            hx = 0;
            hy = 1 + (i - 2 * HW);
        } else {
            hx = HW - 1;
            hy = 1 + (i - 2 * HW - TH);
        }
    }
};

// Pixels of the tw x th tile at (x0, y0) that lie inside the W x H image.
__device__ __forceinline__ int tile_pixels(int W, int H, int tw, int th, int x0, int y0) {
    const int w = W - x0 < tw ? W - x0 : tw;
    const int h = H - y0 < th ? H - y0 : th;
    return w * h;
}

__device__ __forceinline__ void count_px(int64_t *ctr, long long v) {
    atomicAdd((unsigned long long *)ctr, (unsigned long long)v);
}

// Block-wide count of set flags by wave ballots: each wave adds the popcount
// of its ballots once (returned to every thread).
template <int N>
__device__ __forceinline__ int block_count_ballot(const bool (&flag)[N], int *s_red) {
    int c = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) c += __popcll(__ballot(flag[j]));
    __syncthreads();
    if (threadIdx.x == 0) s_red[0] = 0;
    __syncthreads();
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&s_red[0], c);
    __syncthreads();
    return s_red[0];
}

// Block-wide OR of `any` and count of the set `cnt` flags behind a single
// barrier: lane 0 of each wave leaves its wave's ballots in slots[2w] and
// slots[2w + 1] (8 ints), and every thread sums the four.  A previous use of
// the same slots must be separated from this one by a barrier.
template <int N>
__device__ __forceinline__ int2 block_vote(bool any, const bool (&cnt)[N], int *slots) {
    int c = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) c += __popcll(__ballot(cnt[j]));
    const int a = __ballot(any) != 0ull ? 1 : 0;
    const int w = (int)(threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0) {
        slots[2 * w] = a;
        slots[2 * w + 1] = c;
    }
    __syncthreads();
    int2 r = make_int2(0, 0);
#pragma unroll
    for (int i = 0; i < kThreads / 64; ++i) {
        r.x |= slots[2 * i];
        r.y += slots[2 * i + 1];
    }
    return r;
}

// Block-wide OR behind a single barrier (the runtime's block OR takes three):
// lane 0 of each wave writes its wave's ballot to `bank` (4 ints).  Calls
// that follow one another without another barrier in between must alternate
// between two banks: a bank is rewritten only after the barrier of the call
// in between, which every wave reaches after reading it.
__device__ __forceinline__ bool block_any(bool v, int *bank) {
    const int a = __ballot(v) != 0ull ? 1 : 0;
    if ((threadIdx.x & 63) == 0) bank[threadIdx.x >> 6] = a;
    __syncthreads();
    int r = 0;
#pragma unroll
    for (int i = 0; i < kThreads / 64; ++i) r |= bank[i];
    return r != 0;
}

__device__ __forceinline__ long long block_sum_i64(long long v, unsigned long long *s_sum) {
    __syncthreads();
    if (threadIdx.x == 0) *s_sum = 0ull;
    __syncthreads();
    if (v) atomicAdd(s_sum, (unsigned long long)v);
    __syncthreads();
    return (long long)*s_sum;
}

// ---------------------------------------------------------------------------
// Terminal capacities of in-image pixel p (row-major index into the caller's
// arrays) at lambda: seeds are frozen (fg: cs = INF, ct = 0; bg: cs = 0,
// ct = INF), a free pixel has cs = cap_src and ct = cap_snk0 + slope * lambda.
// Values are clamped to [0, INF]; err collects invalid values (bit 0) and
// sink capacities that would exceed INF at the last lambda (bit 1).
// ---------------------------------------------------------------------------
// The raw inputs are read first, for every pixel (a seed's capacities are
// read and ignored), so that a visit's loads are all in flight together.
struct TermIn {
    int sd, cs, c0, sl;
};
__device__ __forceinline__ TermIn load_term(const InstDesc &D, int p) {
    TermIn t;
    t.sd = D.seed ? (int)gp(D.seed)[p] : 0;
    t.cs = gp(D.cap_src)[p];
    t.c0 = gp(D.cap_snk0)[p];
    t.sl = D.slope ? gp(D.slope)[p] : 1;
    return t;
}
__device__ __forceinline__ void terminal_caps(const TermIn &t, long long lam, long long lamL, long long &cs,
                                              long long &ct, int &err) {
    const int sd = t.sd;
    if (sd == 1) {
        cs = kInf;
        ct = 0;
    } else if (sd == 2) {
        cs = 0;
        ct = kInf;
    } else {
        const long long c0 = t.c0;
        const long long sl = t.sl;
        cs = t.cs;
        if (sd != 0) err |= 1;
        if (cs < 0 || cs > kInf || c0 < 0 || sl < 0) err |= 1;
        if (c0 + sl * lamL > kInf) err |= 2;
        ct = c0 + sl * lam;
        cs = cs < 0 ? 0 : (cs > kInf ? kInf : cs);
        ct = ct < 0 ? 0 : (ct > kInf ? kInf : ct);
    }
}

// ---------------------------------------------------------------------------
// kOrient: count the pixels whose source capacity exceeds their sink capacity
// at lambda_0 and those where it is the other way round (paper Sec. 3.2: the
// s-t swap is chosen from these counts), one pass before kInit.
// ---------------------------------------------------------------------------
template <int K, int TW, int TH>
__device__ void orient_tile(const StepParams &P, const InstDesc &D, InstState *S, int tl, int *s_red) {
    using G = Geo<TW, TH>;
    const int tid = threadIdx.x, lx = tid % TW, ly0 = tid / TW;
    const int tx = tl % D.tiles_x, ty = tl / D.tiles_x;
    const int x0 = tx * TW, y0 = ty * TH;
    const int W = D.W, H = D.H;
    const long long lam0 = gp(D.lambdas)[0];
    int err = 0;
    bool pos[G::PPT], neg[G::PPT];
    TermIn tin[G::PPT];
#pragma unroll
    for (int j = 0; j < G::PPT; ++j) {  // pixels outside the image read a clamped position
        const int gx = x0 + lx, gy = y0 + ly0 + j * G::RPI;
        tin[j] = load_term(D, min(gy, H - 1) * W + min(gx, W - 1));
    }
#pragma unroll
    for (int j = 0; j < G::PPT; ++j) {
        const int gx = x0 + lx, gy = y0 + ly0 + j * G::RPI;
        pos[j] = neg[j] = false;
        if (gx >= W || gy >= H) continue;
        long long cs, ct;
        terminal_caps(tin[j], lam0, lam0, cs, ct, err);
        pos[j] = cs > ct;
        neg[j] = cs < ct;
    }
    const int np = block_count_ballot(pos, s_red);
    const int nn = block_count_ballot(neg, s_red);
    if (tid == 0) {
        if (np) atomicAdd(&S->cnt_pos, np);
        if (nn) atomicAdd(&S->cnt_neg, nn);
    }
    (void)P;
}

// ---------------------------------------------------------------------------
// kInit: terminal-arc normalisation at lambda_0 and validation of the inputs.
//   cs, ct per pixel from (seed, cap_src, cap_snk0, slope, lambda_0), exchanged
//   when the instance is solved with source and sink swapped (every n-link
//   then reversed: the residual of p -> q is the capacity of q -> p);
//   the common part m = min(cs, ct) goes straight from s to t: e = cs - m,
//   rt = ct - m; r_k = n-link capacity; inbox cleared.
// ---------------------------------------------------------------------------
template <int K, int TW, int TH>
__device__ void init_tile(const StepParams &P, const InstDesc &D, InstState *S, int tl,
                          int *s_red, unsigned long long *s_sum) {
    using G = Geo<TW, TH>;
    const int tid = threadIdx.x, lx = tid % TW, ly0 = tid / TW;
    const int tx = tl % D.tiles_x, ty = tl / D.tiles_x;
    const int x0 = tx * TW, y0 = ty * TH;
    const int W = D.W, H = D.H, n = D.n;
    const long long lam0 = gp(D.lambdas)[0];
    const long long lamL = gp(D.lambdas)[D.L - 1];
    const bool swap = __builtin_amdgcn_readfirstlane(S->swap) != 0;
    const int32_t nlmax = ((1 << 30) - 1) / K;
    int err = 0;
    long long scs = 0;
    // The pixels in two halves; each half's loads are all issued before any
    // is used (pixels and neighbours outside the image read clamped
    // positions): terminal inputs, n-links and, for an exchanged instance,
    // the reverse n-links.
    constexpr int HP = G::PPT / 2;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        TermIn tin[HP];
        int nl[HP][K], rv[HP][K];
#pragma unroll
        for (int jj = 0; jj < HP; ++jj) {
            const int j = half * HP + jj;
            const int gx = min(x0 + lx, W - 1), gy = min(y0 + ly0 + j * G::RPI, H - 1);
            const int p = gy * W + gx;
            tin[jj] = load_term(D, p);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                nl[jj][k] = gp(D.nlink)[(size_t)k * n + p];
                const int qx = min(max(gx + DXk(k), 0), W - 1), qy = min(max(gy + DYk(k), 0), H - 1);
                rv[jj][k] = swap ? gp(D.nlink)[(size_t)(k ^ 1) * n + qy * W + qx] : 0;
            }
        }
#pragma unroll
        for (int jj = 0; jj < HP; ++jj) {
            const int j = half * HP + jj;
            const int ly = ly0 + j * G::RPI;
            const int gx = x0 + lx, gy = y0 + ly;
            if (gx >= W || gy >= H) continue;
            const int p = gy * W + gx;
            long long cs, ct;
            terminal_caps(tin[jj], lam0, lamL, cs, ct, err);
            if (swap) {
                const long long t = cs;
                cs = ct;
                ct = t;
            }
            const long long m = cs < ct ? cs : ct;
            const int e = (int)(cs - m);
            const int rt = (int)(ct - m);
            scs += cs;
            int rm = (rt > 0 ? kRtBit : 0) | (e > 0 ? kEBit : 0);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int qx = gx + DXk(k), qy = gy + DYk(k);
                const bool on = qx >= 0 && qx < W && qy >= 0 && qy < H;
                int c = nl[jj][k];  // validated here, once per arc
                if (c < 0 || (!on && c != 0)) err |= 1;
                if (c > nlmax) err |= 2;
                if (swap) c = on ? rv[jj][k] : 0;
                if (!on || c < 0) c = 0;
                if (c > nlmax) c = nlmax;
                gp(D.r)[(size_t)k * n + p] = c;
                if (c > 0) rm |= 1 << k;
            }
            gp(D.e)[p] = e;
            gp(D.rt)[p] = rt;
            gp(D.h)[p] = rt > 0 ? 1 : kHInf;
            gp(D.rmask)[p] = (uint16_t)rm;
        }
    }
    for (int i = tid; i < Border<K, TW, TH>::E; i += kThreads)
        gp(D.inbox)[(size_t)tl * Border<K, TW, TH>::E + i] = 0;
    if (tl == 0 && tid < 64) {
        // the schedule: lambda_0 >= 0, non-decreasing (also across the start
        // of a chunk of a longer schedule)
        for (int i = tid; i < D.L; i += 64) {
            const int li = gp(D.lambdas)[i];
            if (li < 0 || (i > 0 && li < gp(D.lambdas)[i - 1])) err |= 1;
        }
        if (tid == 0 && D.check_prev && gp(D.lambdas)[-1] > gp(D.lambdas)[0]) err |= 1;
    }
    const long long tot = block_sum_i64(scs, s_sum);
    if (tid == 0) {
        if (tot) atomicAdd((unsigned long long *)&S->sum_cs, (unsigned long long)tot);
        gp(D.tile_act)[tl] = 0;
        gp(D.tile_cnt)[tl] = 0;
        gp(D.tile_chg)[tl] = 1;
        gp(D.tile_chg)[D.ntiles + tl] = 1;
    }
    if (err) atomicOr(&S->err, err);
    (void)s_red;
}

// ---------------------------------------------------------------------------
// kSweep: tile-local push/relabel iterations in LDS.
//
// The tile's residuals (one record of K words per cell, so that a pixel reads
// all of them at once), excess, sink residuals and heights live in LDS with a
// one-pixel halo.  In every inner iteration each active pixel p (e > 0,
// h < H_INF) pushes d = min(e, r) to the sink when rt > 0 and along
// admissible arcs (h(p) = h(q) + 1), then, if excess is left and no
// admissible arc, relabels to 1 + min h(q) over its residual arcs.  Only the
// active pixels are processed (a small fraction of the tile once the first
// iterations are done).  All residual and excess updates are LDS atomics
// without return: whatever the interleaving of neighbours, every update is
// applied exactly once, a pixel never sends more than the excess and residual
// it read (other threads only add to those), so the bookkeeping stays exact
// and non-negative.  Labels are only a guide here; maximality is
// certified by the exact global relabel.  A push to a halo pixel (another
// tile) lands in the halo cell's word of the reverse arc, i.e. exactly the
// amount handed over; those words go to the neighbours' inboxes at the end.
// ---------------------------------------------------------------------------
template <int K, int TW, int TH, bool GAP>
__device__ void sweep_tile(const StepParams &P, const InstDesc &D, InstState *S, int tl,
                           int iters, int xsw, int32_t *lds, int *s_red) {
    using G = Geo<TW, TH>;
    constexpr int PPT = G::PPT, RPI = G::RPI, HW = G::HW, HH = G::HH, HALO = G::HALO;
    const int tid = threadIdx.x, lx = tid % TW, ly0 = tid / TW;
    const int tx = tl % D.tiles_x, ty = tl / D.tiles_x;
    const int x0 = tx * TW, y0 = ty * TH;
    const int W = D.W, H = D.H, n = D.n;
    const int hcap = n + 1;  // no exact distance to t exceeds n
    int32_t *sh_h = lds;             // [HALO] heights
    int32_t *sh_e = lds + HALO;      // [HALO] excess (tile cells only)
    int32_t *sh_t = lds + 2 * HALO;  // [HALO] sink residuals (tile cells only)
    int32_t *sh_r = lds + 3 * HALO;  // [HALO][K] residuals; halo cells: pushes handed over
    __shared__ int s_nb[9];
    __shared__ uint16_t s_slot[kThreads * PPT + kThreads];  // per wave: its active pixels' cells; then one spare word per thread

    if (tid < 9) s_nb[tid] = 0;
    if (tid == 0) g_and(&gp(D.tile_act)[tl], ~2u);  // about to drain the inbox
    // Every global load of the visit is issued before any is used: the halo
    // cell heights of the neighbour tiles (one ring cell per thread), the
    // state of the thread's pixels, and the tile's inbox words (flow pushed in
    // by neighbour tiles), one or two per thread.  Loads of cells outside the
    // image read a clamped in-image address and are replaced by the defaults.
    bool valid[PPT];
    int e[PPT], rt[PPT], h[PPT], r[PPT][K];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int gx = x0 + lx, gy = y0 + ly0 + j * RPI;
        valid[j] = gx < W && gy < H;
        const int p = min(gy, H - 1) * W + min(gx, W - 1);
        e[j] = gp(D.e)[p];
#pragma unroll
        for (int k = 0; k < K; ++k) r[j][k] = gp(D.r)[(size_t)k * n + p];
        rt[j] = gp(D.rt)[p];
        h[j] = gp(D.h)[p];
    }
    // Gap heuristic: no pixel is labelled `gap` (a level that emptied since
    // the last global relabel), so no pixel labelled above it has a residual
    // path to t while the labels are valid; such pixels stop being active
    // until the next global relabel.  Labels of other tiles may be stale, so
    // this can also stop a pixel that could still reach t: that only delays
    // it (the exact relabel that certifies termination looks at every pixel).
    const int gap = GAP ? __builtin_amdgcn_readfirstlane(
                                __hip_atomic_load(&S->gap, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                          : kHInf;
    static_assert(G::RING <= kThreads, "one halo cell per thread");
    int hx, hy;
    G::ring(min(tid, G::RING - 1), hx, hy);
    const int hc = hy * HW + hx;
    const bool hin = x0 + hx - 1 >= 0 && x0 + hx - 1 < W && y0 + hy - 1 >= 0 && y0 + hy - 1 < H;
    const int hv = gp(D.h)[min(max(y0 + hy - 1, 0), H - 1) * W + min(max(x0 + hx - 1, 0), W - 1)];
    using B = Border<K, TW, TH>;
    constexpr int NBP = (B::E + kThreads - 1) / kThreads;  // inbox words per thread
    GLOBAL int32_t *const inbox = gp(D.inbox) + (size_t)tl * B::E;
    int ibv[NBP];
#pragma unroll
    for (int q = 0; q < NBP; ++q) ibv[q] = ld_agent(&inbox[min(tid + q * kThreads, B::E - 1)]);
    // take exactly what was read: neighbour tiles only ever add to these
    // words (this tile is the only one that takes from them), so subtracting
    // the amount read leaves whatever arrived meanwhile for the next visit,
    // and the subtraction needs no reply
#pragma unroll
    for (int q = 0; q < NBP; ++q) {
        const int i = tid + q * kThreads;
        ibv[q] = i < B::E ? ibv[q] : 0;
        if (ibv[q]) g_add(&inbox[i], -ibv[q]);
    }
    if (tid < G::RING) {
        sh_h[hc] = hin && hv <= gap ? hv : kHInf;
#pragma unroll
        for (int k = 0; k < K; ++k) sh_r[hc * K + k] = 0;  // hand-over words
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int c = (ly0 + j * RPI + 1) * HW + lx + 1;
        sh_e[c] = valid[j] ? e[j] : 0;
        sh_t[c] = valid[j] ? rt[j] : 0;
#pragma unroll
        for (int k = 0; k < K; ++k) sh_r[c * K + k] = valid[j] ? r[j][k] : 0;
        sh_h[c] = valid[j] && h[j] <= gap ? h[j] : kHInf;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NBP; ++q) {
        if (ibv[q]) {
            int bx, by, k;
            B::pair(tid + q * kThreads, bx, by, k);
            const int c = (by + 1) * HW + bx + 1;
            atomicAdd(&sh_e[c], ibv[q]);
            atomicAdd(&sh_r[c * K + k], ibv[q]);
        }
    }
    __syncthreads();

    // Hand pushes into halo cells to the neighbour tiles' inboxes (the word k
    // of halo cell q with q + d_k inside the tile holds what q received) and
    // clear those words; the neighbour tiles are marked for the wake-up below.
    auto flush_halo = [&]() {
        for (int i = tid; i < G::RING; i += kThreads) {
            int hx, hy;
            G::ring(i, hx, hy);
            const int c = hy * HW + hx;
            const int gx = x0 + hx - 1, gy = y0 + hy - 1;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int ix = hx + DXk(k), iy = hy + DYk(k);
                if (ix < 1 || ix > TW || iy < 1 || iy > TH) continue;
                const int v = sh_r[c * K + k];
                if (v > 0 && gx >= 0 && gx < W && gy >= 0 && gy < H) {
                    // the receiving pixel, in the neighbour tile's coordinates
                    const int dtx = hx == 0 ? 0 : (hx == HW - 1 ? 2 : 1);
                    const int dty = hy == 0 ? 0 : (hy == HH - 1 ? 2 : 1);
                    const int bx = dtx == 0 ? TW - 1 : dtx == 2 ? 0 : hx - 1;
                    const int by = dty == 0 ? TH - 1 : dty == 2 ? 0 : hy - 1;
                    const int nt = (ty + dty - 1) * D.tiles_x + tx + dtx - 1;
                    g_add(&gp(D.inbox)[(size_t)nt * B::E + B::index(bx, by, k)], v);
                    sh_r[c * K + k] = 0;
                    s_nb[dty * 3 + dtx] = 1;
                }
            }
        }
    };
    // Mid-visit exchange (short supersteps): flow handed to neighbour tiles
    // that are being swept in the same launch reaches them while they still
    // run, and what they handed here is taken now, so flow can cross several
    // tiles in one superstep.  Taking follows the rule of the visit's start
    // (subtract exactly what was read).
    auto exchange = [&]() {
        __syncthreads();  // every push of the iterations so far is in LDS
        flush_halo();
        int iv[NBP];
#pragma unroll
        for (int q = 0; q < NBP; ++q) iv[q] = ld_agent(&inbox[min(tid + q * kThreads, B::E - 1)]);
#pragma unroll
        for (int q = 0; q < NBP; ++q) {
            const int i = tid + q * kThreads;
            const int v = i < B::E ? iv[q] : 0;
            if (v) {
                g_add(&inbox[i], -v);
                int bx, by, k;
                B::pair(i, bx, by, k);
                const int c = (by + 1) * HW + bx + 1;
                atomicAdd(&sh_e[c], v);
                atomicAdd(&sh_r[c * K + k], v);
            }
        }
        __syncthreads();
    };
    const int xperiod = xsw > 0 ? max(1, iters / (xsw + 1)) : iters + 1;

    // Iterations.  Every pixel belongs to one wave (the PPT pixels of each of
    // its lanes).  Per iteration a wave lists its active pixels (e > 0,
    // h < H_INF) in a slot array of its own, then its lanes take one listed
    // pixel each: sink push, pushes along admissible arcs in arc order, lift
    // if excess is left.  Work is proportional to the active pixels, and
    // waves need no barrier between iterations: every cross-pixel update is
    // an LDS atomic, and a pixel's height and sink residual are written only
    // by its own wave.
    const int lane = tid & 63;
    uint16_t *slot = s_slot + (tid >> 6) * (PPT * 64);
    for (int it = 0; it < iters; ++it) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        int ev[PPT], hv[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int c = (ly0 + j * RPI + 1) * HW + lx + 1;
            ev[j] = sh_e[c];
            hv[j] = sh_h[c];
        }
        int na = 0;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int c = (ly0 + j * RPI + 1) * HW + lx + 1;
            const bool a = (ev[j] > 0) & (hv[j] < kHInf);
            const unsigned long long m = __ballot(a);
            // listed lanes below this one (hardware prefix count), and no
            // branch: every lane writes, the unlisted ones to a word of their own
            const int below_n =
                (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            const int at = a ? (tid >> 6) * (PPT * 64) + na + below_n : kThreads * PPT + tid;
            s_slot[at] = (uint16_t)c;
            na += __popcll(m);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int i = lane; i < na; i += 64) {
            const int c = slot[i];
            int r[K], hq[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                r[k] = sh_r[c * K + k];
                hq[k] = sh_h[c + DYk(k) * HW + DXk(k)];
            }
            const int h = sh_h[c];
            const int rt = sh_t[c];
            // the excess only grew since the listing (only this lane takes it
            // out), so it is still positive
            int ex = sh_e[c];
            const int dt = ex < rt ? ex : rt;
            ex -= dt;
            if (dt) sh_t[c] = rt - dt;
            int pushed = dt;
            const int hm1 = h - 1;
            int mn = kHInf;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int rk = r[k];
                const bool down = hq[k] == hm1;
                const int d = down ? (rk < ex ? rk : ex) : 0;  // residuals are never negative
                ex -= d;
                pushed += d;
                const int cand = rk - d > 0 ? hq[k] + 1 : kHInf;
                mn = cand < mn ? cand : mn;
                if (d) {
                    const int q = c + DYk(k) * HW + DXk(k);
                    atomicSub(&sh_r[c * K + k], d);
                    atomicAdd(&sh_r[q * K + (k ^ 1)], d);
                    // halo cells' excess words are never read: no test needed
                    atomicAdd(&sh_e[q], d);
                }
            }
            if (pushed) atomicSub(&sh_e[c], pushed);
            // excess left means the sink arc and every admissible arc are
            // saturated: lift above the lowest residual neighbour
            if (ex > 0) sh_h[c] = mn >= hcap ? kHInf : mn;
        }
        // progress check every 2 iterations: an iteration in which no wave
        // listed a pixel changed nothing, so the tile is at rest
        if ((it & 1) == 1 || it + 1 == iters) {
            if (!block_any(na > 0, s_red + 16 + 4 * ((it >> 1) & 1))) break;
        }
        if ((it + 1) % xperiod == 0 && it + 1 < iters) exchange();
    }
    __syncthreads();

    // write back
    int active = 0;
    bool killed[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        killed[j] = false;
        if (!valid[j]) continue;
        const int ly = ly0 + j * RPI;
        const int p = (y0 + ly) * W + x0 + lx;
        const int c = (ly + 1) * HW + lx + 1;
        const int h0 = h[j];
        const int e = sh_e[c];
        const int h = sh_h[c];
        active |= e > 0 && h < kHInf;
        if (GAP) {
            // the label histogram follows every stored label below the gap;
            // the level a pixel leaves may empty: a gap below the current one
            killed[j] = h0 > gap && h0 < kHInf;
            if (h0 <= gap && h != h0) {
                if (h0 < D.hsize) {
                    const int was = __hip_atomic_fetch_add(&gp(D.hist)[h0], -1, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                    if (was == 1) atomicMin(&S->gap, h0);
                }
                if (h < D.hsize) g_add(&gp(D.hist)[h], 1);
            }
        }
        const int rt = sh_t[c];
        int rm = (rt > 0 ? kRtBit : 0) | (e > 0 ? kEBit : 0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int r = sh_r[c * K + k];
            gp(D.r)[(size_t)k * n + p] = r;
            if (r > 0) rm |= 1 << k;
        }
        gp(D.e)[p] = e;
        gp(D.rt)[p] = rt;
        gp(D.h)[p] = h;
        gp(D.rmask)[p] = (uint16_t)rm;
    }
    flush_halo();
    // one barrier: the wake-up marks of flush_halo are complete, and the
    // tile's activity (and gap-stopped pixels) are counted
    const int2 vote = block_vote(active != 0, killed, s_red + 8);
    const int tile_active = vote.x, nkill = GAP ? vote.y : 0;
    if (tid < 9 && tid != 4 && s_nb[tid]) {
        const int ntx = tx + (tid % 3) - 1, nty = ty + (tid / 3) - 1;
        if (ntx >= 0 && ntx < D.tiles_x && nty >= 0 && nty < D.tiles_y)
            g_or(&gp(D.tile_act)[nty * D.tiles_x + ntx], 2u);
    }
    if (tid == 0) {
        if (tile_active)
            g_or(&gp(D.tile_act)[tl], 1u);
        else
            g_and(&gp(D.tile_act)[tl], ~1u);
        if (nkill) count_px(&S->gap_kills, nkill);
    }
}

// Whether this tile or one of its neighbours changed a label in the previous pass.
// The nine flags are read unconditionally (a neighbour outside the image
// reads the clamped, in-image position and is ignored), so that the loads
// are in flight together.
__device__ __forceinline__ bool frontier_needs(const InstDesc &D, int tx, int ty, int prev) {
    GLOBAL const uint8_t *chg = gp(D.tile_chg) + (size_t)prev * D.ntiles;
    uint8_t f[9];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int ntx = min(max(tx + dx, 0), D.tiles_x - 1), nty = min(max(ty + dy, 0), D.tiles_y - 1);
            f[(dy + 1) * 3 + dx + 1] = chg[nty * D.tiles_x + ntx];
        }
    bool need = false;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int ntx = tx + dx, nty = ty + dy;
            const bool in = ntx >= 0 && ntx < D.tiles_x && nty >= 0 && nty < D.tiles_y;
            need |= in && f[(dy + 1) * 3 + dx + 1] != 0;
        }
    return need;
}

// ---------------------------------------------------------------------------
// kRelabel: one pass of the exact global relabel (distance to t).
// ---------------------------------------------------------------------------
template <int K, int TW, int TH, bool GAP>
__device__ void relabel_tile(const StepParams &P, const InstDesc &D, InstState *S, int tl,
                             int sub, int xrounds, int32_t *lds, int *s_red) {
    using G = Geo<TW, TH>;
    constexpr int PPT = G::PPT, RPI = G::RPI, HW = G::HW;
    const int tid = threadIdx.x, lx = tid % TW, ly0 = tid / TW;
    const int tx = tl % D.tiles_x, ty = tl / D.tiles_x;
    const int x0 = tx * TW, y0 = ty * TH;
    const int W = D.W, H = D.H, n = D.n;
    const bool first = sub == 0;
    const int cur = sub & 1;  // tile_chg parity written by this pass
    int32_t *sh_d = lds;              // [HALO] labels
    int32_t *sh_in = lds + G::HALO;   // first pass: inflow folded into each tile cell
    int32_t *sh_ib = lds + 2 * G::HALO;  // first pass: arcs whose residual the inflow raised
    int32_t *sh_rm = lds + 3 * G::HALO;  // residual bits of each tile cell (relaxation rounds)
    // Every global load is issued before any is used (cells outside the
    // image read a clamped in-image address and take the defaults): the
    // pixels' residual masks (and labels after the first pass), one halo cell
    // per thread, and in the first pass the tile's inbox words.
    bool valid[PPT];
    uint32_t rm[PPT];
    int d[PPT], d0[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int gx = x0 + lx, gy = y0 + ly0 + j * RPI;
        valid[j] = gx < W && gy < H;
        const int p = min(gy, H - 1) * W + min(gx, W - 1);
        rm[j] = gp(D.rmask)[p];
        d[j] = first ? 0 : gp(D.h)[p];
    }
    int hx, hy;
    G::ring(min(tid, G::RING - 1), hx, hy);
    const bool hin = x0 + hx - 1 >= 0 && x0 + hx - 1 < W && y0 + hy - 1 >= 0 && y0 + hy - 1 < H;
    const int hq = min(max(y0 + hy - 1, 0), H - 1) * W + min(max(x0 + hx - 1, 0), W - 1);
    const int hv = first ? (int)gp(D.rmask)[hq] : gp(D.h)[hq];
    // the tile's active count under the previous labels, read now so that
    // the end of the visit does not wait for it
    const int cnt_prev = (!first && tid == 0) ? gp(D.tile_cnt)[tl] : 0;
    if (first) {
        // fold flow that neighbour tiles pushed into the border pixels (no
        // sweep of this instance runs in the same launch, so nobody else
        // writes the inbox or these residuals meanwhile)
        using B = Border<K, TW, TH>;
        constexpr int NBP = (B::E + kThreads - 1) / kThreads;
        GLOBAL int32_t *const inbox = gp(D.inbox) + (size_t)tl * B::E;
        int ibv[NBP];
#pragma unroll
        for (int q = 0; q < NBP; ++q) ibv[q] = inbox[min(tid + q * kThreads, B::E - 1)];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int c = (ly0 + j * RPI + 1) * HW + lx + 1;
            sh_in[c] = 0;
            sh_ib[c] = 0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NBP; ++q) {
            const int i = tid + q * kThreads;
            const int v = i < B::E ? ibv[q] : 0;
            if (v) {
                int bx, by, k;
                B::pair(i, bx, by, k);
                const int c = (by + 1) * HW + bx + 1;
                inbox[i] = 0;
                g_add(&gp(D.r)[(size_t)k * n + (y0 + by) * W + x0 + bx], v);
                atomicAdd(&sh_in[c], v);
                atomicOr(&sh_ib[c], 1 << k);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int c = (ly0 + j * RPI + 1) * HW + lx + 1;
            const int ein = sh_in[c];
            if (ein && valid[j]) {
                const int p = (y0 + ly0 + j * RPI) * W + x0 + lx;
                g_add(&gp(D.e)[p], ein);
                rm[j] |= (uint32_t)sh_ib[c] | kEBit;
                gp(D.rmask)[p] = (uint16_t)rm[j];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        rm[j] = valid[j] ? rm[j] : 0u;
        d[j] = !valid[j] ? kHInf : first ? ((rm[j] & kRtBit) ? 1 : kHInf) : d[j];
        d0[j] = d[j];
        sh_d[(ly0 + j * RPI + 1) * HW + lx + 1] = d[j];
        sh_rm[(ly0 + j * RPI + 1) * HW + lx + 1] = (int32_t)rm[j];
    }
    if (tid < G::RING)
        sh_d[hy * HW + hx] = !hin ? kHInf : first ? ((hv & kRtBit) ? 1 : kHInf) : hv;
    __syncthreads();
    // After the first pass of a relabel every stored label is an upper bound
    // of the true distance that only decreases, so the tile may publish its
    // improved labels and take newer halo labels written by neighbour tiles
    // during this same launch, several times per visit (exchange rounds).
    // Stale reads only delay convergence.  The first pass keeps one round: its
    // neighbours' stored labels are still those of the previous phase.
    int dpub[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) dpub[j] = d0[j];
    const int rounds = first ? 1 : xrounds;
    for (int round = 0; round < rounds; ++round) {
    // Relaxation rounds; the convergence check (a barrier) runs every 4
    // rounds.  Labels only decrease and every value read is an upper bound of
    // the true distance, so rounds need no barrier between them; a window in
    // which no thread changed a label proves the local fixed point.
    // The rounds work on horizontal strips: thread t owns the 4 consecutive
    // cells (4 (t mod TW/4) .. + 3, t div (TW/4)) of the tile, so the
    // neighbours inside its strip are registers and a round reads only the
    // strip's left and right cells and the rows above and below it from LDS
    // (10 reads at K = 4, 14 at K = 8, against 4K for four scattered cells).
    // The residual bits of the strip come from the LDS copy made below.
    constexpr int SPR = TW / 4;  // strips per row
    const int sy = tid / SPR, sx = 4 * (tid % SPR);
    const int sc = (sy + 1) * HW + sx + 1;  // LDS cell of the strip's first pixel
    uint32_t srm[4];
    int sd[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        srm[j] = (uint32_t)sh_rm[sc + j];
        sd[j] = sh_d[sc + j];
    }
    int ch = 0;
    for (int it = 0; it < P.local_bfs_iters; ++it) {
        // neighbours: up row (sx - 1 .. sx + 4), down row, left and right cells
        int up[6], dn[6];
        const int lf = sh_d[sc - 1], rg = sh_d[sc + 4];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            if (K == 4 && (i == 0 || i == 5)) {
                up[i] = dn[i] = kHInf;  // corners: diagonal arcs only
                continue;
            }
            up[i] = sh_d[sc - HW - 1 + i];
            dn[i] = sh_d[sc + HW - 1 + i];
        }
        // branch-free: every label is rewritten (only its owner writes it) as
        // min(d, 1 + min over residual arcs of the neighbour's label), taken
        // as 1 + min(d - 1, neighbour label or H_INF - 1 where the arc is
        // saturated): one select per arc; a result never exceeds H_INF.
        // The strip's cells are taken in order, left to right in even rounds
        // and right to left in odd ones, each seeing the label its strip
        // neighbour got earlier in the same round, so a distance crosses
        // the whole strip in one round in the direction of the pass.
        auto relax = [&](int j) {
            int nb[8];
            nb[0] = j < 3 ? sd[j + 1] : rg;  // (+1, 0)
            nb[1] = j > 0 ? sd[j - 1] : lf;  // (-1, 0)
            nb[2] = dn[j + 1];               // (0, +1)
            nb[3] = up[j + 1];               // (0, -1)
            nb[4] = dn[j + 2];               // (+1, +1)
            nb[5] = up[j];                   // (-1, -1)
            nb[6] = dn[j];                   // (-1, +1)
            nb[7] = up[j + 2];               // (+1, -1)
            int mn = sd[j] - 1;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int vk = ((srm[j] >> k) & 1u) ? nb[k] : kHInf - 1;
                mn = vk < mn ? vk : mn;
            }
            ch |= mn + 1 < sd[j];
            sd[j] = mn + 1;
        };
#pragma unroll
        for (int j = 0; j < 4; ++j) relax(j);
#pragma unroll
        for (int j = 0; j < 4; ++j) sh_d[sc + j] = sd[j];
        if ((it & 3) == 3 || it + 1 == P.local_bfs_iters) {
            if (!block_any(ch != 0, s_red + 16 + 4 * ((it >> 2) & 1))) break;
            ch = 0;
        }
    }
    __syncthreads();
    // back to the load layout
#pragma unroll
    for (int j = 0; j < PPT; ++j) d[j] = sh_d[(ly0 + j * RPI + 1) * HW + lx + 1];
    if (round + 1 == rounds) break;
    // publish, then take the neighbours' newer labels
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int ly = ly0 + j * RPI;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx < W && gy < H && d[j] < dpub[j]) {
            st_agent(&gp(D.h)[gy * W + gx], d[j]);
            dpub[j] = d[j];
        }
    }
    int got = 0;
    for (int i = tid; i < G::RING; i += kThreads) {
        int hx, hy;
        G::ring(i, hx, hy);
        const int gx = x0 + hx - 1, gy = y0 + hy - 1;
        if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;
        const int v = ld_agent(&gp(D.h)[gy * W + gx]);
        if (v < sh_d[hy * HW + hx]) {
            sh_d[hy * HW + hx] = v;
            got = 1;
        }
    }
    if (!block_any(got != 0, s_red + 24)) break;
    }
    int changed = first ? 1 : 0;
    bool act[PPT], one[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int ly = ly0 + j * RPI;
        const int gx = x0 + lx, gy = y0 + ly;
        act[j] = (rm[j] & kEBit) && d[j] < kHInf;  // rm = 0 outside the image
        one[j] = first && d[j] == 1;
        if (gx >= W || gy >= H) continue;
        if (first || d[j] != d0[j]) changed = 1;
        if (first || d[j] != dpub[j]) gp(D.h)[gy * W + gx] = d[j];
        // gap heuristic: the label histogram follows every change after the
        // first pass (which sets every label to 1 or H_INF and clears it)
        if (GAP && !first && d[j] != d0[j]) {
            if (d0[j] < D.hsize) g_add(&gp(D.hist)[d0[j]], -1);
            if (d[j] < D.hsize) g_add(&gp(D.hist)[d[j]], 1);
        }
    }
    if (GAP && first) {
        // this tile's share of the histogram starts at zero; the count of
        // label-1 pixels goes to hist[1] once every first-pass tile is done
        for (int i = tid; i < TW * TH; i += kThreads) gp(D.hist)[(size_t)tl * (TW * TH) + i] = 0;
        const int ones = block_count_ballot(one, s_red);
        if (tid == 0 && ones) atomicAdd(&S->hist1, ones);
    }
    const int2 vote = block_vote(changed != 0, act, s_red + 8);
    const int tchg = vote.x, tcnt = vote.y;
    if (tid == 0) {
        gp(D.tile_chg)[(size_t)cur * D.ntiles + tl] = (uint8_t)(tchg ? 1 : 0);
        const int delta = first ? tcnt : tcnt - cnt_prev;
        gp(D.tile_cnt)[tl] = tcnt;
        if (delta) atomicAdd(&S->active, delta);
        if (tchg) atomicOr(&S->changed, 1);
        gp(D.tile_act)[tl] = tcnt > 0 ? 1u : 0u;
    }
}

// ---------------------------------------------------------------------------
// kCut for an instance solved with source and sink exchanged.  The minimal
// source set of the original graph is the set of pixels that can reach the
// exchanged sink in the residual graph of the maximum preflow (the minimal
// sink side of the exchanged graph), i.e. those with a finite label after the
// converged relabel: one pass, no reachability search.  The pass also sums
// the excess (F = sum cs - sum e in either orientation) and raises the
// exchanged source capacities to the next lambda: the increase of a free
// pixel's source arc first cancels against its sink residual, the rest
// becomes excess; the preflow stays valid.  The added capacity joins sum cs
// once this lambda's flow has been taken.
// ---------------------------------------------------------------------------
template <int K, int TW, int TH>
__device__ void cut_tile_swapped(const StepParams &P, const InstDesc &D, InstState *S, int tl, int kk,
                                 int *s_red, unsigned long long *s_sum) {
    using G = Geo<TW, TH>;
    constexpr int PPT = G::PPT, RPI = G::RPI;
    const int tid = threadIdx.x, lx = tid % TW, ly0 = tid / TW;
    const int tx = tl % D.tiles_x, ty = tl / D.tiles_x;
    const int x0 = tx * TW, y0 = ty * TH;
    const int W = D.W, H = D.H, n = D.n;
    GLOBAL uint8_t *mask = gp(D.masks) + (size_t)kk * n;
    const int dlam = kk + 1 < D.L ? gp(D.lambdas)[kk + 1] - gp(D.lambdas)[kk] : 0;
    int hv[PPT], rmv[PPT], ev[PPT], rtv[PPT], sdv[PPT], slv[PPT];
    bool valid[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int gx = x0 + lx, gy = y0 + ly0 + j * RPI;
        valid[j] = gx < W && gy < H;
        const int p = min(gy, H - 1) * W + min(gx, W - 1);
        hv[j] = gp(D.h)[p];
        rmv[j] = gp(D.rmask)[p];
        ev[j] = gp(D.e)[p];
        rtv[j] = gp(D.rt)[p];
        sdv[j] = 0;
        slv[j] = 1;
        if (dlam > 0) {
            if (D.seed) sdv[j] = gp(D.seed)[p];
            if (D.slope) slv[j] = gp(D.slope)[p];
        }
    }
    long long se = 0, sraise = 0;
    int act = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (!valid[j]) continue;
        const int p = (y0 + ly0 + j * RPI) * W + x0 + lx;
        mask[p] = hv[j] < kHInf ? 1 : 0;
        if (rmv[j] & kEBit) se += ev[j];
        const int sl = sdv[j] == 0 ? slv[j] : 0;
        if (dlam > 0 && sl > 0) {
            const int inc = (int)((long long)sl * dlam);  // <= INF: checked at init
            sraise += inc;
            const int d = inc < rtv[j] ? inc : rtv[j];
            const int nrt = rtv[j] - d, ne = ev[j] + (inc - d);
            gp(D.rt)[p] = nrt;
            gp(D.e)[p] = ne;
            const int rm = (rmv[j] & ~(kRtBit | kEBit)) | (nrt > 0 ? kRtBit : 0) | (ne > 0 ? kEBit : 0);
            if (rm != rmv[j]) gp(D.rmask)[p] = (uint16_t)rm;
            act |= ne > 0 && hv[j] < kHInf;
        }
    }
    const long long tse = block_sum_i64(se, s_sum);
    const long long tra = block_sum_i64(sraise, s_sum);
    // The next lambda starts from these labels (exchanged instances skip the
    // relabel there): the tiles with a pixel made active by the raise are the
    // sweep's work (every other tile has none: the relabel that ended this
    // lambda left no active pixel).
    const int tact = block_any(act != 0, s_red + 28) ? 1 : 0;
    if (tid == 0) {
        if (tact) g_or(&gp(D.tile_act)[tl], 1u);
        gp(D.tile_chg)[tl] = 0;  // the cut is complete after this pass
        if (tse) atomicAdd((unsigned long long *)&S->sum_e, (unsigned long long)tse);
        if (tra) atomicAdd((unsigned long long *)&S->sum_raise, (unsigned long long)tra);
    }
    (void)P;
}

// ---------------------------------------------------------------------------
// kCut: one pass of the forward residual reachability from excess pixels.
// The first pass also sums the excess (for F) and raises the sink residuals
// to the next lambda (warm start).
// ---------------------------------------------------------------------------
template <int K, int TW, int TH>
__device__ void cut_tile(const StepParams &P, const InstDesc &D, InstState *S, int tl, int sub,
                         int kk, int xrounds, int32_t *lds, int *s_red, unsigned long long *s_sum) {
    using G = Geo<TW, TH>;
    constexpr int PPT = G::PPT, RPI = G::RPI, HW = G::HW;
    const int tid = threadIdx.x, lx = tid % TW, ly0 = tid / TW;
    const int tx = tl % D.tiles_x, ty = tl / D.tiles_x;
    const int x0 = tx * TW, y0 = ty * TH;
    const int W = D.W, H = D.H, n = D.n;
    const bool first = sub == 0;
    const int cur = sub & 1;  // tile_chg parity written by this pass
    GLOBAL uint8_t *mask = gp(D.masks) + (size_t)kk * n;
    // one LDS word per cell: the residual bits, and bit 15 = reached
    constexpr int kReached = 1 << 15;
    int32_t *sh_w = lds;
    const bool raise = first && kk + 1 < D.L;
    const int dlam = raise ? gp(D.lambdas)[kk + 1] - gp(D.lambdas)[kk] : 0;
    // Every global load is issued before any is used (cells outside the image
    // read a clamped in-image address and take the defaults).
    int m[PPT], m0[PPT], rmv[PPT], ev[PPT], rtv[PPT], sdv[PPT], slv[PPT];
    bool valid[PPT];
    long long se = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int gx = x0 + lx, gy = y0 + ly0 + j * RPI;
        valid[j] = gx < W && gy < H;
        const int p = min(gy, H - 1) * W + min(gx, W - 1);
        rmv[j] = gp(D.rmask)[p];
        m[j] = 0;
        ev[j] = rtv[j] = sdv[j] = 0;
        slv[j] = 1;
        if (first) {
            ev[j] = gp(D.e)[p];
            if (dlam > 0) {
                rtv[j] = gp(D.rt)[p];
                if (D.seed) sdv[j] = gp(D.seed)[p];
                if (D.slope) slv[j] = gp(D.slope)[p];
            }
        } else {
            m[j] = mask[p];
        }
    }
    int hx, hy;
    G::ring(min(tid, G::RING - 1), hx, hy);
    const bool hin = x0 + hx - 1 >= 0 && x0 + hx - 1 < W && y0 + hy - 1 >= 0 && y0 + hy - 1 < H;
    const int hq = min(max(y0 + hy - 1, 0), H - 1) * W + min(max(x0 + hx - 1, 0), W - 1);
    const int hrm = gp(D.rmask)[hq];
    const int hmk = first ? ((hrm & kEBit) ? 1 : 0) : mask[hq];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (!valid[j]) {
            rmv[j] = 0;
            m[j] = 0;
        } else if (first) {
            m[j] = (rmv[j] & kEBit) ? 1 : 0;
            if (m[j]) se += ev[j];
            // raise the sink residuals to the next lambda (warm start)
            const int sl = sdv[j] == 0 ? slv[j] : 0;
            if (dlam > 0 && sl > 0) {
                const int p = (y0 + ly0 + j * RPI) * W + x0 + lx;
                const int nrt = rtv[j] + sl * dlam;
                gp(D.rt)[p] = nrt;
                if (nrt > 0 && !(rmv[j] & kRtBit)) gp(D.rmask)[p] = (uint16_t)(rmv[j] | kRtBit);
            }
        }
        m0[j] = m[j];
        sh_w[(ly0 + j * RPI + 1) * HW + lx + 1] = rmv[j] | (m[j] ? kReached : 0);
    }
    if (tid < G::RING) sh_w[hy * HW + hx] = hin ? (hrm | (hmk ? kReached : 0)) : 0;
    __syncthreads();
    // Exchange rounds as in the relabel pass: after the first pass every stored
    // reached bit is final once set, so newer bits of neighbour tiles written
    // during this launch can be taken up within the visit.
    int mpub[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) mpub[j] = m0[j];
    const int rounds = first ? 1 : xrounds;
    for (int round = 0; round < rounds; ++round) {
    // Reachability rounds, convergence checked every 4 rounds: reached bits
    // only get set, so rounds need no barrier between them.
    int ch = 0;
    for (int it = 0; it < P.local_bfs_iters; ++it) {
        int v[PPT][K];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int c = (ly0 + j * RPI + 1) * HW + lx + 1;
#pragma unroll
            for (int k = 0; k < K; ++k) v[j][k] = sh_w[c + DYk(k) * HW + DXk(k)];
        }
        // branch-free; a pixel outside the image is never reached: its
        // neighbours have no residual arc towards it
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            int reach = 0;
#pragma unroll
            for (int k = 0; k < K; ++k)  // q = p + d_k reaches p if q is reached and r(q -> p) > 0
                reach |= (v[j][k] >> (k ^ 1)) & (v[j][k] >> 15);
            const int nm = m[j] | (reach & 1);
            ch |= nm ^ m[j];
            m[j] = nm;
            sh_w[(ly0 + j * RPI + 1) * HW + lx + 1] = rmv[j] | (nm << 15);
        }
        if ((it & 3) == 3 || it + 1 == P.local_bfs_iters) {
            if (!block_any(ch != 0, s_red + 16 + 4 * ((it >> 2) & 1))) break;
            ch = 0;
        }
    }
    if (round + 1 == rounds) break;
    // publish, then take the neighbours' newer reached bits
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int ly = ly0 + j * RPI;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx < W && gy < H && m[j] && !mpub[j]) {
            st_agent(&mask[gy * W + gx], (uint8_t)1);
            mpub[j] = 1;
        }
    }
    int got = 0;
    for (int i = tid; i < G::RING; i += kThreads) {
        int hx, hy;
        G::ring(i, hx, hy);
        const int gx = x0 + hx - 1, gy = y0 + hy - 1;
        if (gx < 0 || gx >= W || gy < 0 || gy >= H) continue;
        const int c = hy * HW + hx;
        if (!(sh_w[c] & kReached) && ld_agent(&mask[gy * W + gx])) {
            sh_w[c] |= kReached;
            got = 1;
        }
    }
    if (!block_any(got != 0, s_red + 24)) break;
    }
    int changed = first ? 1 : 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int ly = ly0 + j * RPI;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= W || gy >= H) continue;
        if (first || m[j] != m0[j]) changed = 1;
        if (first || m[j] != mpub[j]) mask[gy * W + gx] = (uint8_t)m[j];
    }
    const int tchg = block_any(changed != 0, s_red + 28) ? 1 : 0;
    long long tse = 0;
    if (first) tse = block_sum_i64(se, s_sum);
    if (tid == 0) {
        gp(D.tile_chg)[(size_t)cur * D.ntiles + tl] = (uint8_t)(tchg ? 1 : 0);
        if (tchg) atomicOr(&S->changed, 1);
        if (tse) atomicAdd((unsigned long long *)&S->sum_e, (unsigned long long)tse);
    }
}

// ---------------------------------------------------------------------------
// Phase machine of every instance of the work list (one thread each), run
// after the tile work of every superstep.
// ---------------------------------------------------------------------------
// Returns whether the instance is still running afterwards.
__device__ bool control_one(const StepParams &P, int w) {
    const int i = P.wl_ident ? w : P.wl_slot[w];
    // The state and the descriptor fields used here are read in one batch:
    // this kernel runs alone after the tile kernels of the superstep, whose
    // writes it sees at the launch boundary.
    InstState S = P.st[i];
    const InstDesc *Dp = &P.desc[i];
    const int L = Dp->L;
    int64_t *flows = Dp->flows;
    int32_t *status_out = Dp->status;
    int ph = S.phase;
    if (ph == kIdle || ph == kDone) return false;
    S.steps += 1;
    bool done = false;
    int status = PMF_OK;
    switch (ph) {
        case kOrient:
            S.swap = P.orientation == kOrientMoreSink ? S.cnt_neg > S.cnt_pos : S.cnt_pos > S.cnt_neg;
            ph = kInit;
            S.sub = 0;
            break;
        case kInit:
            if (S.err) {
                done = true;
                status = (S.err & 1) ? PMF_EINVAL : PMF_EOVERFLOW;
            } else {
                ph = kRelabel;
                S.sub = 0;
                S.active = 0;
            }
            break;
        case kRelabel:
            S.passes += 1;
            // gap heuristic: the first pass has cleared the histogram and
            // counted the pixels it labelled 1
            if (P.gap && S.sub == 0) gp(Dp->hist)[1] = S.hist1;
            if (S.sub > 0 && !S.changed) {
                S.relabels += 1;
                ph = S.active == 0 ? kCut : kSweep;
                S.sub = 0;
            } else if (P.relabel_passes > 0 && S.sub + 1 >= P.relabel_passes && S.active > 0) {
                // cut short: the pixels labelled so far hold upper bounds of
                // their distances and there is work for the sweep; pixels
                // still at H_INF wait for a later relabel.  Only a relabel
                // run to its fixed point may end the solve.
                S.relabels += 1;
                ph = kSweep;
                S.sub = 0;
            } else {
                S.sub += 1;
            }
            break;
        case kSweep:
            S.sweeps += 1;
            if (++S.sub >= P.sweeps_per_relabel || !S.listed) {
                ph = kRelabel;
                S.sub = 0;
                S.active = 0;
            }
            break;
        case kCut:
            S.passes += 1;
            // an exchanged instance's cut takes one pass (it reads the labels)
            if ((S.sub > 0 || S.swap) && !S.changed) {
                const int k = S.k;
                gp(flows)[k] = S.sum_cs - S.sum_e;
                S.sum_e = 0;
                S.sum_cs += S.sum_raise;  // the next lambda's source capacity (exchanged instances)
                S.sum_raise = 0;
                S.k = k + 1;
                if (k + 1 >= L) {
                    done = true;
                } else if (S.swap) {
                    // exchanged: the raise only took sink residual away, so no
                    // distance shrank and the converged labels stay valid
                    // lower bounds: the next lambda sweeps from them at once
                    ph = kSweep;
                    S.sub = 0;
                } else {
                    ph = kRelabel;
                    S.sub = 0;
                    S.active = 0;
                }
            } else {
                S.sub += 1;
            }
            break;
    }
    S.changed = 0;
    if (ph == kRelabel && S.sub == 0) {
        // a relabel starts: its first pass rebuilds the label histogram, and
        // no level is known to be empty until a sweep empties one
        S.gap = kHInf;
        S.hist1 = 0;
    }
    if (!done && S.steps >= P.max_steps) {
        done = true;
        status = PMF_ETIMEOUT;
    }
    if (done) {
        if (status != PMF_OK) {
            const int from = status == PMF_ETIMEOUT ? S.k : 0;
            for (int k = from; k < L; ++k) gp(flows)[k] = -1;
        }
        if (status_out) *gp(status_out) = status;
        ph = kDone;
        const int at = atomicAdd(P.ring_count, 1);
        P.ring[at % P.ring_cap] = i;
    }
    S.phase = ph;
    P.st[i] = S;
    return ph != kDone;
}

// Append `value` to `list` for every lane whose `want` is set: one atomic per
// wave on the list counter, lanes packed in lane order.
__device__ __forceinline__ void wave_append(bool want, int2 *list, int32_t *count, int2 value) {
    const unsigned long long m = __ballot(want);
    if (m == 0ull) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, leader);
    if (want) list[base + __popcll(m & ((1ull << lane) - 1ull))] = value;
}

// Work compaction, one workgroup per instance of the work list: the tiles
// that need a sweep (instance sweeping, pixels active or inflow pending) and
// the tiles that need a relabel / cut / init pass (first pass of a phase, or a
// change in the 3x3 tile neighbourhood during the previous pass) go to four
// lists (sweep K=4, sweep K=8, pass K=4, pass K=8) as {instance slot, tile}
// pairs.  Skipped pass tiles record "no change" for the current pass here, as
// a processed tile would.  The tile kernels rely on these tests: a listed tile
// is in range, its instance in the listed phase (phases change only in the
// control kernel), a listed sweep tile has work, a listed pass tile needs
// the pass.  Every listed tile is visited exactly once by the tile work that
// follows, so the pixel-visit statistics of that work are counted here, by
// the instance's own workgroup, rather than by every visit.
__device__ void compact_instance(const StepParams &P, int w) {
    __shared__ int s_vote[8];
    const int slot = P.wl_ident ? w : __builtin_amdgcn_readfirstlane(P.wl_slot[w]);
    const InstState *S = &P.st[slot];
    const int phase = __builtin_amdgcn_readfirstlane(S->phase);
    const int sub = __builtin_amdgcn_readfirstlane(S->sub);
    const int swap = __builtin_amdgcn_readfirstlane(S->swap);  // read with the phase: the kind of the visits
    if (phase != kSweep && phase != kInit && phase != kOrient && phase != kRelabel && phase != kCut) return;
    const InstDesc D = load_desc(P.desc, slot);
    const bool is8 = D.K == 8;
    int2 *lists = reinterpret_cast<int2 *>(P.lists);
    int2 *sl = lists + (is8 ? 1 : 0) * (size_t)P.list_cap;
    int2 *pl = lists + (is8 ? 3 : 2) * (size_t)P.list_cap;
    int32_t *sc = P.list_count + (is8 ? 1 : 0), *pc = P.list_count + (is8 ? 3 : 2);
    int nsw = 0;
    const int tw = D.tile_w, th = (kThreads * 4) / tw;
    int npx = 0;  // pixels of the tiles this thread listed
    __syncthreads();  // a previous call's vote has been read (persistent launches compact several instances)
    for (int t0 = 0; t0 < D.ntiles; t0 += kThreads) {
        const int tl = t0 + (int)threadIdx.x;
        bool sw = false, bf = false;
        if (tl < D.ntiles) {
            if (phase == kSweep) {
                sw = (gp(D.tile_act)[tl] & 3u) != 0u;
            } else if (phase == kInit || phase == kOrient || sub == 0) {
                bf = true;
            } else {
                const int tx = tl % D.tiles_x, ty = tl / D.tiles_x;
                bf = frontier_needs(D, tx, ty, (sub & 1) ^ 1);
                if (!bf) gp(D.tile_chg)[(size_t)(sub & 1) * D.ntiles + tl] = 0;
            }
        }
        const int2 en = make_int2(slot, tl);
        wave_append(sw, sl, sc, en);
        wave_append(bf, pl, pc, en);
        nsw |= sw;
        if (sw || bf) npx += tile_pixels(D.W, D.H, tw, th, (tl % D.tiles_x) * tw, (tl / D.tiles_x) * th);
    }
    // one barrier: whether a tile was listed to sweep (a sweeping instance
    // with no tile to sweep is at rest: the control kernel then starts its
    // relabel at once) and the listed pixels (at most 2^31 per instance)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) npx += __shfl_xor(npx, off);
    const int wv = (int)(threadIdx.x >> 6);
    const bool wany = __ballot(nsw != 0) != 0ull;
    if ((threadIdx.x & 63) == 0) {
        s_vote[2 * wv] = wany ? 1 : 0;
        s_vote[2 * wv + 1] = npx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int any = 0;
        long long v = 0;
#pragma unroll
        for (int i = 0; i < kThreads / 64; ++i) {
            any |= s_vote[2 * i];
            v += s_vote[2 * i + 1];
        }
        InstState *Sw = &P.st[slot];
        Sw->listed = any;
        if (v) {
            const int kind = phase == kSweep ? kPxSweep
                             : phase == kRelabel ? kPxRelabel
                             : phase == kOrient ? kPxOrient
                             : phase == kInit ? (swap ? kPxInitX : kPxInit)
                                              : (swap ? kPxCutX : kPxCut);
            int64_t *ctr = kind == kPxSweep     ? &Sw->px_sweep
                           : kind == kPxRelabel ? &Sw->px_relabel
                           : kind == kPxOrient  ? &Sw->px_orient
                           : kind == kPxInit    ? &Sw->px_init
                           : kind == kPxInitX   ? &Sw->px_init_x
                           : kind == kPxCut     ? &Sw->px_cut
                                                : &Sw->px_cut_x;
            count_px(ctr, v);  // no reply awaited
            if (P.kpx) count_px(&P.kpx[kind], v);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_compact(StepParams P) { compact_instance(P, (int)blockIdx.x); }

// Item i of a list, the same for every thread of the workgroup (scalar registers).
__device__ __forceinline__ int2 list_item(const StepParams &P, int which, int i) {
    const int2 en = reinterpret_cast<const int2 *>(P.lists)[(size_t)which * P.list_cap + i];
    return make_int2(__builtin_amdgcn_readfirstlane(en.x), __builtin_amdgcn_readfirstlane(en.y));
}

// Tile work of one superstep for one connectivity: the items of sweep list
// `ws` and of pass list `wp` (-1: none).  An instance is either sweeping or
// in a pass, so the two kinds of items never touch the same instance and may
// run side by side.  Workgroup b takes items of its XCD's eighth of each list
// (b & 7 picks the eighth: consecutive items are neighbouring tiles of one
// image, which then share an L2), round robin over the XCD's workgroups.
template <int K, int TW, int TH, bool GAP>
__device__ void tile_work(const StepParams &P, int ws, int wp, int32_t *lds, int *s_red, unsigned long long *s_sum) {
    const int ns = ws >= 0 ? P.list_count[ws] : 0;
    const int np = wp >= 0 ? P.list_count[wp] : 0;
    const int x = (int)(blockIdx.x & 7), stride = (int)(gridDim.x >> 3), first = (int)(blockIdx.x >> 3);
    const int es = (ns + 7) >> 3, ep = (np + 7) >> 3;
    const int s_lo = x * es, s_n = max(0, min(ns, s_lo + es) - s_lo);
    const int p_lo = x * ep, p_n = max(0, min(np, p_lo + ep) - p_lo);
    // a short superstep (few tiles in a kind of list) is latency bound: its
    // visits may run longer at no cost in width
    const bool short_sweeps = P.list_count[0] + P.list_count[1] < P.tail_tiles;
    const int iters = short_sweeps ? P.tail_inner_iters : P.inner_iters;
    const int xsw = short_sweeps ? P.tail_sweep_exchanges : 0;
    const int xrounds =
        P.list_count[2] + P.list_count[3] < P.tail_tiles ? P.tail_exchange_rounds : P.exchange_rounds;
    for (int i = first; i < s_n + p_n; i += stride) {
        __syncthreads();  // the previous item's LDS is no longer in use
        if (i < s_n) {
            const int2 en = list_item(P, ws, s_lo + i);
            const InstDesc D = load_desc(P.desc, en.x);
            sweep_tile<K, TW, TH, GAP>(P, D, &P.st[en.x], en.y, iters, xsw, lds, s_red);
        } else {
            const int2 en = list_item(P, wp, p_lo + i - s_n);
            InstState *S = &P.st[en.x];
            const int phase = S->phase, sub = S->sub, kk = S->k, swap = S->swap;
            const InstDesc D = load_desc(P.desc, en.x);
            const int tl = en.y;
            if (phase == kInit)
                init_tile<K, TW, TH>(P, D, S, tl, s_red, s_sum);
            else if (phase == kOrient)
                orient_tile<K, TW, TH>(P, D, S, tl, s_red);
            else if (phase == kRelabel)
                relabel_tile<K, TW, TH, GAP>(P, D, S, tl, sub, xrounds, lds, s_red);
            else if (swap)
                cut_tile_swapped<K, TW, TH>(P, D, S, tl, kk, s_red, s_sum);
            else
                cut_tile<K, TW, TH>(P, D, S, tl, sub, kk, xrounds, lds, s_red, s_sum);
        }
    }
}

// GAP: the gap heuristic's label histogram is kept (a variant of its own, so
// that the default build carries none of its registers).  TIMED: the same
// code under a name of its own for the launches of timing mode, so that a
// profiler's kernel trace reports exactly the launches that mode times.
// The 4-connected kernel is held to 128 VGPRs: four waves per SIMD, which its
// LDS also allows (four workgroups per CU).
template <int K, int TW, int TH, bool GAP, bool TIMED = false>
__global__ __launch_bounds__(kThreads, K == 4 ? 4 : 1) void k_step(StepParams P, int ws, int wp) {
    __shared__ int32_t lds[(3 + K) * (TW + 2) * (TH + 2)];  // sweep layout; passes use 4 planes
    __shared__ int s_red[32];  // [0]: block_count_ballot, [8..15]: block_vote, [16..31]: block_any
    __shared__ unsigned long long s_sum;
    tile_work<K, TW, TH, GAP>(P, ws, wp, lds, s_red, &s_sum);
}

__global__ __launch_bounds__(kThreads) void k_control(StepParams P) {
    const int w = (int)(blockIdx.x * kThreads + threadIdx.x);
    if (w < P.nwl) (void)control_one(P, w);
    if (blockIdx.x == 0 && threadIdx.x < 4) {
        if (P.trace_lists) P.trace_lists[threadIdx.x] = P.list_count[threadIdx.x];
        // keep this superstep's list sizes (read by the timing mode), then
        // clear them: the next superstep compacts afresh
        P.list_count[4 + threadIdx.x] = P.list_count[threadIdx.x];
        P.list_count[threadIdx.x] = 0;
    }
}

// ---------------------------------------------------------------------------
// Persistent supersteps.  When few tiles have work the superstep is latency
// bound and its three launches cost more than their work; k_persist then runs
// supersteps back to back inside one cooperative launch (every workgroup
// resident): compaction, tile work of both connectivities and the phase
// machine, separated by grid-wide barriers.  It leaves when every instance of
// the work list is done, when a superstep listed more than `exit_tiles` tiles
// (wide again: separate launches spread them better), after `max_steps`
// supersteps, or when a barrier wait exceeds its time limit (then it raises
// the abort word and every workgroup returns; the host reports an error).
// Barrier words (int32, after the list counters): [0] arrivals, [1]
// generation, [2] abort, [3] supersteps run by the last launch, [4..5] running
// instances counted by the control phase of even / odd supersteps.
// ---------------------------------------------------------------------------
constexpr int kBarWords = 16;                    // offset of the barrier words in the counter block
constexpr long long kBarrierTicks = 100000000;   // 1 s of the 100 MHz constant clock

// The workgroup's writes are complete once its barrier has passed (a
// workgroup barrier waits for the stores of every wave); one thread then
// makes them visible device-wide (release fence), arrives, and waits for the
// generation to change with relaxed loads (no cache invalidation while it
// spins), then one acquire fence makes the other workgroups' writes visible
// here.  Returns false (in every thread) when the wait was abandoned.
__device__ bool grid_barrier(int32_t *bar, unsigned nblocks, int *s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        uint32_t *arrive = reinterpret_cast<uint32_t *>(bar);
        uint32_t *gen = reinterpret_cast<uint32_t *>(bar + 1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t at = __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (at == nblocks) {
            // every other workgroup has arrived (and released its writes)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const long long t0 = wall_clock64();
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (__hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    ok = 0;
                    break;
                }
                if (wall_clock64() - t0 > kBarrierTicks) {
                    __hip_atomic_store(bar + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// The superstep parameters of a persistent launch live in device memory (the
// host copies them there before the launch) and are read with scalar loads.
__device__ __forceinline__ StepParams load_params(const StepParams *src) {
    static_assert(sizeof(StepParams) % 4 == 0, "parameters read in 4-byte words");
    const __attribute__((address_space(4))) uint32_t *w =
        (const __attribute__((address_space(4))) uint32_t *)src;
    StepParams P;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&P);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(StepParams) / 4); ++i) dst[i] = w[i];
    return P;
}

// Persistent kernels come in three forms: for work lists of 4-connected
// instances only (KSET 4), of 8-connected ones only (KSET 8), both inlined
// into the kernel; and for mixed lists (KSET 12), whose phases are separate
// (not inlined) functions so that each gets the registers it needs rather
// than the sum of both connectivities.  The sweep and pass layouts use the
// launch's dynamic LDS.
extern __shared__ int32_t persist_lds[];

template <int K, int TW, int TH>
__device__ __attribute__((noinline)) void persist_work(const StepParams *Pg) {
    __shared__ int s_red[32];  // [0]: block_count_ballot, [8..15]: block_vote, [16..31]: block_any
    __shared__ unsigned long long s_sum;
    const StepParams P = load_params(Pg);
    tile_work<K, TW, TH, false>(P, K == 4 ? 0 : 1, K == 4 ? 2 : 3, persist_lds, s_red, &s_sum);
}

__device__ __attribute__((noinline)) void persist_compact(const StepParams *Pg) {
    const StepParams P = load_params(Pg);
    for (int w = (int)blockIdx.x; w < P.nwl; w += (int)gridDim.x) compact_instance(P, w);
}

// Phase machine of the instances of this workgroup's share; whether one of
// them is still running.
__device__ __forceinline__ int control_share(const StepParams &P) {
    int run = 0;
    for (int w = (int)(blockIdx.x * kThreads + threadIdx.x); w < P.nwl; w += (int)gridDim.x * kThreads)
        run |= control_one(P, w) ? 1 : 0;
    return run;
}

__device__ __attribute__((noinline)) int persist_control(const StepParams *Pg) {
    const StepParams P = load_params(Pg);
    return control_share(P);
}

template <int TW, int TH, int KSET>
__global__ __launch_bounds__(kThreads) void k_persist(const StepParams *Pg, int max_steps, int exit_tiles) {
    __shared__ int s_ok;
    __shared__ int s_red[32];  // [0]: block_count_ballot, [8..15]: block_vote, [16..31]: block_any
    __shared__ unsigned long long s_sum;
    const StepParams P = load_params(Pg);
    int32_t *bar = P.ring_count + kBarWords;
    const unsigned G = gridDim.x;
    for (int step = 0; step < max_steps; ++step) {
        // compaction: the instances of the work list, round robin over the workgroups
        if (KSET == 12) {
            persist_compact(Pg);
        } else {
            for (int w = (int)blockIdx.x; w < P.nwl; w += (int)G) compact_instance(P, w);
        }
        if (!grid_barrier(bar, G, &s_ok)) return;
        // tile work; the running count of the next superstep starts at zero
        // (its readers, after the previous superstep, are all past the barrier)
        if (blockIdx.x == 0 && threadIdx.x == 0) bar[4 + ((step + 1) & 1)] = 0;
        if (KSET == 4) {
            tile_work<4, TW, TH, false>(P, 0, 2, persist_lds, s_red, &s_sum);
        } else if (KSET == 8) {
            tile_work<8, TW, TH, false>(P, 1, 3, persist_lds, s_red, &s_sum);
        } else {
            persist_work<4, TW, TH>(Pg);
            __syncthreads();
            persist_work<8, TW, TH>(Pg);
        }
        if (!grid_barrier(bar, G, &s_ok)) return;
        // phase machine of every instance; the list sizes are kept and cleared
        const int run = KSET == 12 ? persist_control(Pg) : control_share(P);
        if (__syncthreads_or(run) && threadIdx.x == 0) atomicAdd(&bar[4 + (step & 1)], 1);
        if (blockIdx.x == 0 && threadIdx.x < 4) {
            P.list_count[4 + threadIdx.x] = P.list_count[threadIdx.x];
            P.list_count[threadIdx.x] = 0;
        }
        if (!grid_barrier(bar, G, &s_ok)) return;
        if (blockIdx.x == 0 && threadIdx.x == 0) bar[3] = step + 1;
        const int running = __hip_atomic_load(&bar[4 + (step & 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int listed = P.list_count[4] + P.list_count[5] + P.list_count[6] + P.list_count[7];
        if (running == 0 || listed > exit_tiles) break;
    }
}

// Nested masks to one byte per pixel: the number of lambdas whose minimal
// source side holds the pixel (the sets shrink as lambda grows, so mask k is
// level > k).
__global__ __launch_bounds__(kThreads) void k_levels(const uint8_t *masks, int L, int n, uint8_t *out,
                                                     int accumulate) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= n) return;
    int c = accumulate ? out[p] : 0;
    for (int k = 0; k < L; ++k) c += masks[(size_t)k * n + p];
    out[p] = (uint8_t)c;
}

int launch_levels(const uint8_t *masks, int L, int n, uint8_t *out, bool accumulate, void *stream) {
    hipLaunchKernelGGL(k_levels, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, (hipStream_t)stream,
                       masks, L, n, out, accumulate ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// meta layout: first[n_user + 1], flow_off[n_user], L[n_user] (int64)
__global__ __launch_bounds__(kThreads) void k_finalize(const int32_t *sub_status, const int64_t *meta,
                                                       int n_user, int64_t *flows, int32_t *status_out) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n_user) return;
    const int64_t *first = meta, *off = meta + n_user + 1, *len = meta + 2 * n_user + 1;
    bool inval = false, over = false, tout = false;
    for (int64_t c = first[i]; c < first[i + 1]; ++c) {
        const int st = sub_status[c];
        inval |= st == PMF_EINVAL;
        over |= st == PMF_EOVERFLOW;
        tout |= st == PMF_ETIMEOUT;
    }
    const int st = inval ? PMF_EINVAL : over ? PMF_EOVERFLOW : tout ? PMF_ETIMEOUT : PMF_OK;
    if (inval || over)
        for (int64_t k = 0; k < len[i]; ++k) flows[off[i] + k] = -1;
    if (status_out) status_out[i] = st;
}

int launch_finalize(const int32_t *sub_status, const int64_t *meta, int n_user, int64_t *flows,
                    int32_t *status_out, void *stream) {
    hipLaunchKernelGGL(k_finalize, dim3((n_user + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       (hipStream_t)stream, sub_status, meta, n_user, flows, status_out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Workgroups of a list-driven launch, a multiple of 8: several times what the
// device holds at once (about 1024 of the 4-connected kernel, 768 of the
// 8-connected one), so that a compute unit whose items ran short takes up
// another workgroup's: the dispatcher balances the superstep's uneven visits
// (a workgroup with no item left exits at once).
static int list_grid(int tiles) { return 8 * ((std::min(tiles, 4096) + 7) / 8); }

// One tile-work launch of connectivity K over sweep list ws and pass list wp
// (no launch when the work list has no tile of that connectivity).  With
// start / stop events the launch records the kernel's own start and end
// (hipExtLaunchKernel), so timing excludes the dispatch gaps around it.
template <int K, int TW, int TH>
static bool step_launch(const StepParams &p, hipStream_t s, int ws, int wp, hipEvent_t start = nullptr,
                        hipEvent_t stop = nullptr) {
    const int tiles = K == 4 ? p.t4_count : p.t8_count;
    if (!tiles) return false;
    const dim3 g(list_grid(tiles)), b(kThreads);
    const bool timed = start || stop;  // plain launches otherwise (they are also captured into graphs)
    if (p.gap) {
        if (timed)
            hipExtLaunchKernelGGL((k_step<K, TW, TH, true, true>), g, b, 0, s, start, stop, 0, p, ws, wp);
        else
            hipLaunchKernelGGL((k_step<K, TW, TH, true>), g, b, 0, s, p, ws, wp);
    } else {
        if (timed)
            hipExtLaunchKernelGGL((k_step<K, TW, TH, false, true>), g, b, 0, s, start, stop, 0, p, ws, wp);
        else
            hipLaunchKernelGGL((k_step<K, TW, TH, false>), g, b, 0, s, p, ws, wp);
    }
    return true;
}

// The tile-work launches of one kind (both connectivities): the first records
// `start`, the last `stop`.
template <int TW, int TH>
static int step_pair(const StepParams &p, hipStream_t s, int ws4, int wp4, int ws8, int wp8, hipEvent_t start,
                     hipEvent_t stop) {
    const bool a = p.t4_count > 0, b = p.t8_count > 0;
    int n = 0;
    if (a) n += step_launch<4, TW, TH>(p, s, ws4, wp4, start, b ? nullptr : stop);
    if (b) n += step_launch<8, TW, TH>(p, s, ws8, wp8, a ? nullptr : start, stop);
    return n;
}

template <int TW, int TH>
static int launch_tw(const StepParams &p, hipStream_t s, void *const *ev, bool split) {
    const dim3 block(kThreads);
    if (p.ntiles == 0) return 0;
    hipEvent_t *e = (hipEvent_t *)ev;
    hipLaunchKernelGGL(k_compact, dim3(p.nwl), block, 0, s, p);
    int n;
    if (split) {
        // sweeps and passes as separate launches (timed apart)
        n = step_pair<TW, TH>(p, s, 0, -1, 1, -1, e ? e[0] : nullptr, e ? e[1] : nullptr);
        n += step_pair<TW, TH>(p, s, -1, 2, -1, 3, e ? e[2] : nullptr, e ? e[3] : nullptr);
    } else {
        n = step_pair<TW, TH>(p, s, 0, 2, 1, 3, e ? e[0] : nullptr, e ? e[1] : nullptr);
    }
    const dim3 cg((p.nwl + kThreads - 1) / kThreads);
    if (e)
        hipExtLaunchKernelGGL(k_control, cg, block, 0, s, e[4], e[5], 0, p);
    else
        hipLaunchKernelGGL(k_control, cg, block, 0, s, p);
    return n;
}

int resident_workgroups(int K, int tile_w) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e;
    if (tile_w == 64)
        e = K == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_step<8, 64, 16, false>, kThreads, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_step<4, 64, 16, false>, kThreads, 0);
    else
        e = K == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_step<8, 32, 32, false>, kThreads, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_step<4, 32, 32, false>, kThreads, 0);
    return e == hipSuccess ? per * cus : 0;
}

// Dynamic LDS of a persistent launch: the sweep layout of its connectivity
// (the 8-connected one for mixed lists).
static unsigned persist_lds_bytes(int tile_w, int kset) {
    const int tw = tile_w == 64 ? 64 : 32, th = 1024 / tw, K = kset == 4 ? 4 : 8;
    return (unsigned)((3 + K) * (tw + 2) * (th + 2) * 4);
}

template <int TW, int TH>
static const void *persist_fn(int kset) {
    return kset == 4 ? (const void *)k_persist<TW, TH, 4>
                     : kset == 8 ? (const void *)k_persist<TW, TH, 8> : (const void *)k_persist<TW, TH, 12>;
}

int persist_workgroups(int tile_w, int kset) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const void *fn = tile_w == 64 ? persist_fn<64, 16>(kset) : persist_fn<32, 32>(kset);
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kThreads, persist_lds_bytes(tile_w, kset));
    return e == hipSuccess ? per * cus : 0;
}

int launch_persist(const StepParams *p_dev, int tile_w, int kset, int grid, int max_steps, int exit_tiles,
                   void *stream) {
    if (grid < 8 || grid % 8 != 0 || max_steps < 1 || !p_dev) return -1;
    if (kset != 4 && kset != 8 && kset != 12) return -1;
    const StepParams *a = p_dev;
    void *args[] = {(void *)&a, (void *)&max_steps, (void *)&exit_tiles};
    const void *fn = tile_w == 64 ? persist_fn<64, 16>(kset) : persist_fn<32, 32>(kset);
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kThreads), args,
                                                    persist_lds_bytes(tile_w, kset), (hipStream_t)stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    return 0;
}

int launch_superstep(const StepParams &p, int tile_w, void *stream, void *const *events, bool split) {
    hipStream_t s = (hipStream_t)stream;
    const int n = tile_w == 64 ? launch_tw<64, 16>(p, s, events, split) : launch_tw<32, 32>(p, s, events, split);
    return hipGetLastError() == hipSuccess ? n : -1;
}

}  // namespace pmf
