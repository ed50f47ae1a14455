// Internal data structures shared by the host side of libpmf and its kernels.
//
// Device state of one instance (one image/seed problem, its lambda schedule):
//   r      int32 [K][n]  residual capacity of the arc p -> p + d_k
//   e      int32 [n]     excess of p (flow in minus flow out)
//   rt     int32 [n]     residual capacity of the arc p -> t
//   h      int32 [n]     height (distance label); H_INF = "cannot reach t"
//   inbox  int32 [ntiles][border_words]  flow pushed into a border pixel p
//                        from p + d_k in another tile, not yet folded into e
//                        and r: one word per (border pixel, arc leaving the
//                        tile) pair
//   rmask  uint16 [n]    bit k: r_k > 0, bit 8: rt > 0, bit 9: e > 0
//   masks  uint8 [L][n]  minimal source side for every lambda
//   hist   int32 [ntiles * TW * TH]  (gap heuristic only) number of pixels
//                        whose stored label is each value below the size
// All pixel planes are row-major with pitch W, 256-byte aligned.
#pragma once

#include <stdint.h>

namespace pmf {

constexpr int32_t kInf = 1 << 30;       // terminal capacity of seeds
constexpr int32_t kHInf = 1 << 30;      // height meaning "no residual path to t"
constexpr int kThreads = 256;           // workgroup size (4 wave64)
constexpr int kRtBit = 1 << 8;
constexpr int kEBit = 1 << 9;

// Inbox words of one tw x th tile with K-connectivity: each border row holds
// one word per pixel for every arc that leaves the tile through it (1 arc at
// K = 4, 3 at K = 8), each border column likewise.
constexpr int border_words(int K, int tw, int th) { return (K == 4 ? 2 : 6) * (tw + th); }

enum Phase : int32_t {
    kIdle = 0,   // slot unused
    kInit = 1,   // t-link normalisation + validation (one pass)
    kRelabel = 2,// global relabel: exact BFS distances to t (passes until stable)
    kSweep = 3,  // tile-local push/relabel sweeps
    kCut = 4,    // forward residual reachability from excess pixels (passes until stable)
    kDone = 5,
    kOrient = 6, // count pixels with cs > ct and cs < ct at lambda_0 (one pass, before kInit)
};

// Orientation policies (pmf_options.orientation): solve the graph as given, or
// with source and sink exchanged and every arc reversed (same flow value, and
// the minimal source set of the original is read off the reversed graph's
// converged labels).
enum Orientation : int32_t {
    kOrientAsGiven = 0,
    kOrientMoreSink = 1,    // exchange when more pixels have cs < ct than cs > ct
    kOrientMoreSource = 2,  // exchange when more pixels have cs > ct than cs < ct
    kOrientExchange = 3,    // always exchange
};

struct alignas(16) InstDesc {
    int32_t W, H, K, n;
    int32_t tiles_x, tiles_y, ntiles, tile0;
    int32_t L, slot_id;
    int32_t check_prev;  // lambdas[-1] belongs to the same schedule: check it too
    int32_t tile_w;      // tile width in pixels (tiles hold 1024 pixels)
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
    uint32_t *tile_act;  // [ntiles] bit 0: active pixels, bit 1: inbox pending
    uint8_t *tile_chg;   // [2][ntiles] a label changed in the pass of that parity
    int32_t *tile_cnt;   // [ntiles] active pixels under the current labels
    int32_t *hist;       // gap heuristic: pixels per label value (null when off)
    int32_t hsize;       // entries of hist (ntiles * TW * TH); larger labels are not counted
    int32_t pad2;
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
    int64_t px_init, px_sweep, px_relabel, px_cut;  // pixel visits per phase
    int32_t swap;     // 1: solved with source and sink exchanged (decided once per instance)
    int32_t cnt_pos;  // kOrient: pixels with cs > ct at lambda_0
    int32_t cnt_neg;  // kOrient: pixels with cs < ct at lambda_0
    int32_t listed;   // the last compaction listed a tile of this instance to sweep
    int64_t sum_raise;  // exchanged instances: source capacity added for the next lambda
    int64_t px_orient, px_init_x, px_cut_x;  // pixel visits: orientation count, exchanged init and cut
    int32_t gap;      // gap heuristic: lowest label level found empty since the last relabel (kHInf: none)
    int32_t hist1;    // gap heuristic: pixels labelled 1 by the first pass of the current relabel
    int64_t gap_kills;  // pixels found above an empty level by the sweeps (statistics)
};

struct StepParams {
    InstDesc *desc;             // [nslots]
    InstState *st;              // [nslots]
    const int32_t *wl_slot;     // work list: slots of the live instances, 4-connected first
    int32_t nwl;                // entries of wl_slot
    int32_t wl_ident;           // 1: wl_slot[w] == w for every entry (the kernels then skip the lookup)
    int32_t *ring;              // completion ring: slots in order of completion
    int32_t *ring_count;        // completions so far (ring index = count % ring_cap)
    int32_t ring_cap;
    int32_t list_cap;           // capacity of each compacted list (>= ntiles)
    int32_t *lists;             // [4][list_cap] {slot, tile} pairs: to sweep (K=4, K=8), to pass (K=4, K=8)
    int32_t *list_count;        // [4] entries of each list in this superstep, [4..7] those of the last one
    int32_t ntiles;
    int32_t t4_count;           // tiles of the 4-connected instances of the work list
    int32_t t8_count;           // tiles of the 8-connected ones
    int32_t nslots;
    int32_t inner_iters;
    int32_t sweeps_per_relabel;
    int32_t local_bfs_iters;
    int32_t exchange_rounds;
    int32_t tail_tiles;         // lists shorter than this use the two settings below
    int32_t tail_inner_iters;
    int32_t tail_exchange_rounds;
    int32_t tail_sweep_exchanges;  // short supersteps: mid-visit flow exchanges of a sweep visit
    int32_t relabel_passes;     // cap on the passes of a relabel that leaves active pixels (0 = none)
    int32_t orientation;        // Orientation policy
    int32_t gap;                // 1: gap heuristic (every descriptor then has a hist array)
    int64_t max_steps;
    int32_t *trace_lists;       // timing mode: the control kernel copies the 4 list sizes here (may be null)
    int64_t *kpx;               // timing mode: pixel visits of the listed tiles by kind (may be null)
};

// Kinds of tile work (index into StepParams::kpx and pmf_stats::kernel_px).
enum PxKind : int { kPxSweep = 0, kPxRelabel, kPxCut, kPxInit, kPxOrient, kPxInitX, kPxCutX, kPxKinds };

// Enqueue one superstep (compaction, tile work and control kernels) over
// every tile (defined in pmf_kernels.hip).  The sweeps and the relabel / cut
// / init passes of a connectivity share one launch.  With `events` (6
// hipEvent_t) the launches record their kernels' own start and end: events
// 0 / 1 the tile work (with `split`: the sweeps, the sweeps and passes then
// being separate launches), 2 / 3 the passes (split only), 4 / 5 the control
// kernel.  Returns the number of tile-work kernels launched, or -1 on a
// launch error.
int launch_superstep(const StepParams &p, int tile_w, void *stream, void *const *events = nullptr,
                     bool split = false);

// Workgroups of the tile kernel of connectivity K that the current device
// holds at once (0 if the runtime cannot tell).
int resident_workgroups(int K, int tile_w);

// Persistent supersteps (one cooperative launch of `grid` workgroups, a
// multiple of 8 no larger than persist_workgroups(), reading the parameters
// from a device copy p_dev): up to max_steps
// supersteps, leaving early when no instance of the work list is running or
// when a superstep listed more than exit_tiles tiles.  The counter block
// after the list counters holds the barrier words: [16] arrivals, [17]
// generation, [18] abort (a barrier wait gave up: the state is not usable),
// [19] supersteps run.  Returns 0, or -1 if the launch was refused.
// kset: 4 or 8 when every instance of the work list has that connectivity,
// 12 for a mixed list.  Not for the gap heuristic.
constexpr int kBarAbort = 18, kBarSteps = 19;
int persist_workgroups(int tile_w, int kset);
int launch_persist(const StepParams *p_dev, int tile_w, int kset, int grid, int max_steps, int exit_tiles,
                   void *stream);

// out[p] (+)= number of the L masks that hold pixel p (n pixels).
int launch_levels(const uint8_t *masks, int L, int n, uint8_t *out, bool accumulate, void *stream);

// Merge the statuses of the lambda chunks of each caller instance:
// user i owns chunks [first[i], first[i+1]) and flows [flow_off[i], +L[i]).
// The merged status is EINVAL, else EOVERFLOW, else ETIMEOUT, else OK; an
// invalid instance gets flows -1 throughout.
int launch_finalize(const int32_t *sub_status, const int64_t *meta, int n_user, int64_t *flows,
                    int32_t *status_out, void *stream);

}  // namespace pmf
