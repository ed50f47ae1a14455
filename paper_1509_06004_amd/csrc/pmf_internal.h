// Internal data structures shared by the host side of libpmf and its kernels.
//
// Device state of one instance (one image/seed problem, its lambda schedule):
//   r      int32 [K][n]  residual capacity of the arc p -> p + d_k
//   e      int32 [n]     excess of p (flow in minus flow out)
//   rt     int32 [n]     residual capacity of the arc p -> t
//   h      int32 [n]     height (distance label); H_INF = "cannot reach t"
//   inbox  int32 [K][n]  flow pushed into p from p + d_k by another tile,
//                        not yet folded into e and r (cross-tile pushes)
//   rmask  uint16 [n]    bit k: r_k > 0, bit 8: rt > 0, bit 9: e > 0
//   masks  uint8 [L][n]  minimal source side for every lambda
// All planes are row-major with pitch W, 256-byte aligned.
#pragma once

#include <stdint.h>

namespace pmf {

constexpr int32_t kInf = 1 << 30;       // terminal capacity of seeds
constexpr int32_t kHInf = 1 << 30;      // height meaning "no residual path to t"
constexpr int kThreads = 256;           // workgroup size (4 wave64)
constexpr int kRtBit = 1 << 8;
constexpr int kEBit = 1 << 9;

enum Phase : int32_t {
    kIdle = 0,   // slot unused
    kInit = 1,   // t-link normalisation + validation (one pass)
    kRelabel = 2,// global relabel: exact BFS distances to t (passes until stable)
    kSweep = 3,  // tile-local push/relabel sweeps
    kCut = 4,    // forward residual reachability from excess pixels (passes until stable)
    kDone = 5,
};

struct alignas(16) InstDesc {
    int32_t W, H, K, n;
    int32_t tiles_x, tiles_y, ntiles, tile0;
    int32_t L, slot_id;
    int32_t pad0, pad1;
    const int32_t *lambdas;
    const int32_t *nlink;
    const int32_t *cap_src;
    const int32_t *cap_snk0;
    const int32_t *slope;  // may be null: slope 1
    const uint8_t *seed;   // may be null: all free
    int32_t *r;
    int32_t *e;
    int32_t *rt;
    int32_t *h;
    int32_t *inbox;
    uint16_t *rmask;
    uint8_t *masks;
    int64_t *flows;   // L entries (caller memory)
    int32_t *status;  // 1 entry (caller memory), may be null
};

struct alignas(16) InstState {
    int32_t phase;
    int32_t k;        // index of the lambda being solved
    int32_t sub;      // pass / sweep counter inside the phase
    int32_t err;      // bit 0: invalid value, bit 1: headroom exceeded
    int32_t changed;  // a tile changed a label during the last pass
    int32_t active;   // active pixels (e > 0, h < H_INF) under the current labels
    int32_t sweeps;   // sweep supersteps (statistics)
    int32_t relabels; // completed global relabels (statistics)
    int64_t sum_cs;   // total source capacity (F = sum_cs - sum of excess)
    int64_t sum_e;    // total excess at the end of a lambda
    int64_t steps;    // supersteps spent (budget)
    int64_t passes;   // relaxation passes (statistics)
};

struct StepParams {
    InstDesc *desc;
    InstState *st;
    const int32_t *tile_slot;   // [ntiles] instance slot of each tile
    const int32_t *tile_local;  // [ntiles] tile index inside its instance
    uint32_t *tile_act;         // [ntiles] bit 0 active pixels, bit 1 inbox pending
    uint8_t *tile_chg;          // [2][ntiles] label changed in pass (parity)
    int32_t *tile_cnt;          // [ntiles] active pixels under current labels
    uint32_t *arrive;           // arrival counter of the last-workgroup pattern
    int32_t *ndone;             // instances finished (read by the host)
    int64_t *counters;          // [4] sweep visits, bfs tile passes, relabels, steps
    int32_t ntiles;
    int32_t per_xcd;            // ceil(ntiles / 8)
    int32_t nslots;
    int32_t inner_iters;
    int32_t sweeps_per_relabel;
    int32_t local_bfs_iters;
    int64_t max_steps;
};

// Launch one superstep over every tile (defined in pmf_kernels.hip).
int launch_superstep(const StepParams &p, int tile_w, void *stream);
int max_lds_bytes(int tile_w);

}  // namespace pmf
