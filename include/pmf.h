/*
 * pmf.h -- C ABI of libpmf: exact parametric maximum flow / minimum s-t cut on
 * 4- and 8-connected image grids, solved on one AMD Instinct MI355X (gfx950).
 *
 * The problem (paper Sec. 2 and 2.1): every pixel is a vertex linked to the
 * source s and the sink t by terminal arcs (data terms) and to its neighbours
 * by smoothness arcs.  Seeds are pixels frozen to a label: foreground seeds
 * are tied to s, background seeds to t, both with capacity PMF_INF.  The sink
 * capacity of a free pixel grows linearly with a parameter lambda (the
 * monotone parametric case, whose optimal source sets are nested), and a
 * preset, non-decreasing lambda schedule is solved (the "lambda-schedule" of
 * Sec. 2.1).  For every lambda of every instance the library returns
 *   - the maximum flow value F(lambda) (= minimum cut cost, Ford-Fulkerson),
 *   - the inclusion-minimal minimum-cut source side S_min(lambda) as a mask.
 * Results are exact integers and do not depend on launch configuration.
 *
 * Many instances of different sizes are solved in one call; they are packed
 * into the same device launches (the device-side counterpart of the paper's
 * lambda- and seed-supergraphs, Sec. 3.1).
 *
 * Conventions
 *   - Direction k has offset (DX[k], DY[k]) with
 *       DX = { 1,-1, 0, 0, 1,-1,-1, 1 },  DY = { 0, 0, 1,-1, 1,-1, 1,-1 };
 *     k ^ 1 is the opposite direction.  K = 4 uses directions 0..3, K = 8 all.
 *   - All planes are row-major, pixel p = y * W + x, no padding.
 *   - "device" pointers are HIP device memory on the handle's device; the
 *     caller owns them.  No function takes ownership of caller memory.
 *   - Every function returns PMF_OK (0) or a positive PMF_E* code; no C++
 *     exception crosses this interface.
 */
#ifndef PMF_H
#define PMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PMF_INF (1 << 30) /* capacity of the terminal arcs of seeds */

enum pmf_status {
    PMF_OK = 0,
    PMF_EINVAL = 1,     /* bad argument or bad capacity value            */
    PMF_EOVERFLOW = 2,  /* capacities exceed the int32 headroom (below)  */
    PMF_ENOMEM = 3,     /* device memory or workspace too small          */
    PMF_EDEVICE = 4,    /* HIP runtime error                             */
    PMF_ETIMEOUT = 5,   /* superstep budget exhausted for an instance    */
    PMF_ENOTSOLVED = 6, /* no completed solve to read from               */
    PMF_ERANGE = 7,     /* instance or lambda index out of range         */
    PMF_EBUSY = 8,      /* no free slot; retry after results are released */
    PMF_ELIMIT = 9      /* batch larger than PMF_NOALLOC_BYTES (no-allocation solve) */
};

/* Solver options.  Fill with pmf_default_options(); every field is a tuning
 * knob that changes speed, never results. */
typedef struct pmf_options {
    int32_t tile_w;             /* tile width in pixels: 32 or 64 (0 = default)     */
    int32_t tile_h;             /* tile height: tile_w * tile_h = 1024 (0 = default) */
    int32_t inner_iters;        /* push/relabel iterations per tile visit            */
    int32_t sweeps_per_relabel; /* sweep supersteps between global relabels          */
    int32_t local_bfs_iters;    /* bound on relaxation rounds between halo reads     */
    int32_t steps_per_sync;     /* supersteps per host completion check              */
    int64_t max_supersteps;     /* per-instance budget; exceeding it = PMF_ETIMEOUT  */
    int32_t use_graph;          /* 1: replay supersteps from a captured hipGraph     */
    int32_t order;              /* 0: FIFO packing order, 1: LPT (largest first)     */
    int64_t mem_budget;         /* bytes the library may allocate (0 = no limit)     */
    int32_t max_slots;          /* instance slots of a serving session (0 = 4096)    */
    int32_t timing;             /* 1: no graph; time every launch with HIP events;   */
                                /*   2: the same, with sweeps and passes launched   */
                                /*   separately (timed apart)                       */
    int32_t lambda_chunk;       /* pmf_solve_batch: lambdas per device instance.     */
                                /*   1 = every lambda solved from scratch, all in   */
                                /*   parallel; >= L = one warm-started chain; 0 =   */
                                /*   the smallest chunk whose state fits in memory  */
    int32_t exchange_rounds;    /* relabel/cut passes: halo re-reads per tile visit  */
    int32_t tail_tiles;         /* a superstep whose sweep (pass) list holds fewer   */
                                /*   tiles than this is latency bound: its sweeps   */
                                /*   use tail_inner_iters, its relabel / cut passes */
                                /*   tail_exchange_rounds (0 = never)               */
    int32_t tail_inner_iters;
    int32_t tail_exchange_rounds;
    int32_t relabel_passes;     /* a global relabel that still leaves active pixels */
                                /*   after this many passes hands over to the sweep */
                                /*   before its fixed point (0 = never); a relabel  */
                                /*   that certifies termination always converges    */
    int32_t orientation;        /* s-t swap (paper Sec. 3.2): solve each instance   */
                                /*   as given (0), with source and sink exchanged   */
                                /*   and arcs reversed when more pixels have cs < ct */
                                /*   than cs > ct at lambda_0 (1, the paper's rule), */
                                /*   when more have cs > ct (2), or always (3).     */
                                /*   Results are the same in every case.            */
    int32_t gap;                /* 1: gap heuristic between global relabels         */
                                /*   (Cherkassky-Goldberg): a per-instance count of */
                                /*   pixels per label, kept by the relabel passes   */
                                /*   and the sweeps; when a level empties, the      */
                                /*   pixels above it cannot reach the sink and stop */
                                /*   being active until the next global relabel.    */
                                /*   0: off.  Costs 4 bytes of device memory per    */
                                /*   pixel.                                         */
    int32_t persist_tiles;      /* once a superstep lists fewer tiles than this,    */
                                /*   supersteps run back to back inside one         */
                                /*   cooperative (persistent) launch, separated by  */
                                /*   grid-wide barriers, until the lists grow past  */
                                /*   twice this, every instance is done, or the     */
                                /*   host polls (0 = never; not with gap = 1)       */
    int32_t persist_wgs;        /* workgroups of that launch (0 = one per compute   */
                                /*   unit; at most what the device holds at once)   */
    int32_t tail_sweep_exchanges; /* short supersteps: a sweep visit hands its      */
                                /*   cross-tile pushes to the neighbour tiles and   */
                                /*   takes theirs this many times during the visit  */
                                /*   (0 = only at its end)                          */
} pmf_options;

/* One (image, seed) problem and its lambda schedule.  All pointers are device
 * pointers that must stay valid until the solve that uses them has returned
 * (pmf_solve_batch) or the instance has completed (serving calls).
 *
 *   nlink     int32 [K][H][W]  capacity of the arc p -> p + d_k, 0 <= c <= PMF_NLINK_MAX(K);
 *                              must be 0 where the neighbour is off the grid.
 *                              Instances of one image may share this pointer.
 *   cap_src   int32 [H][W]     source capacity of free pixels, 0..PMF_INF
 *   cap_snk0  int32 [H][W]     sink capacity of free pixels at lambda = 0, >= 0
 *   snk_slope int32 [H][W]     d(sink capacity)/d(lambda) of free pixels, >= 0;
 *                              NULL means 1 everywhere
 *   seed      uint8 [H][W]     0 free, 1 foreground (cs = INF, ct = 0),
 *                              2 background (cs = 0, ct = INF); NULL = all free
 *   lambdas   int32 [L]        non-decreasing, >= 0; duplicates allowed
 *
 * Headroom: every per-pixel quantity of the solver is an int32.  The call
 * fails with PMF_EOVERFLOW unless cap_snk0 + snk_slope * lambdas[L-1] <= INF
 * and every n-link capacity is at most PMF_NLINK_MAX(K), which keeps excess
 * (<= INF + K * max n-link) below 2^31. */
typedef struct pmf_instance {
    int32_t W, H, K, L;
    const int32_t *nlink;
    const int32_t *cap_src;
    const int32_t *cap_snk0;
    const int32_t *snk_slope;
    const uint8_t *seed;
    const int32_t *lambdas;
} pmf_instance;

#define PMF_NLINK_MAX(K) ((int32_t)(((1 << 30) - 1) / (K)))

typedef struct pmf_handle pmf_handle;

/* Per-handle counters of the last solve (or of the session so far). */
typedef struct pmf_stats {
    int64_t supersteps;       /* device launches of the superstep kernel            */
    int64_t sweep_visits;     /* tile visits that ran push/relabel iterations       */
    int64_t global_relabels;  /* completed global relabels (all instances)          */
    int64_t bfs_passes;       /* tile-parallel relaxation passes (relabel + cut)    */
    int64_t host_syncs;       /* host completion checks                             */
    int64_t device_bytes;     /* bytes of device memory held by the handle          */
    int64_t device_ns;        /* GPU time of the superstep launches (HIP events)    */
    int64_t px_init;          /* pixel visits per phase, summed over tiles:         */
    int64_t px_sweep;         /*   init, push/relabel sweeps, global-relabel passes */
    int64_t px_relabel;       /*   and cut passes (the unit of the algorithmic      */
    int64_t px_cut;           /*   byte counts)                                     */
    int64_t work_ns;          /* with opt.timing: GPU time of the tile-work         */
                              /*   launches (sweeps and passes),                    */
    int64_t sweep_ns;         /*   with opt.timing = 2 that of the sweeps and of    */
    int64_t pass_ns;          /*   the init/relabel/cut passes apart,               */
    int64_t control_ns;       /*   and that of the phase-machine kernel             */
    int64_t work_launches;    /* launches of the tile-work kernels                  */
    int64_t px_orient;        /* pixel visits of the orientation count, of the init */
    int64_t px_init_x;        /*   and of the cut passes of exchanged instances     */
    int64_t px_cut_x;         /*   (not in px_init / px_cut)                        */
    int64_t gap_kills;        /* pixels the gap heuristic stopped (options.gap)     */
    int64_t persist_launches; /* persistent launches, the supersteps they ran and,  */
    int64_t persist_supersteps; /* with opt.timing, their GPU time                  */
    int64_t persist_ns;
    int64_t kernel_px[16];    /* with opt.timing: pixel visits of the tile-work     */
                              /*   launches ([0..6]) and of the persistent launches */
                              /*   ([8..14]) by kind: sweep, relabel pass, cut      */
                              /*   pass, init, orientation count, exchanged init,   */
                              /*   exchanged cut                                    */
} pmf_stats;

/* Fill *opt with defaults. */
void pmf_default_options(pmf_options *opt);

/* Create a handle bound to the current HIP device and to `stream` (a
 * hipStream_t; NULL = the default stream).  `workspace` (device memory of
 * `ws_bytes` bytes, caller-owned) is used for all solver state when non-NULL;
 * otherwise the library allocates with hipMalloc, within opt->mem_budget.
 * opt may be NULL (defaults).  Errors: PMF_EINVAL (bad option or NULL out),
 * PMF_EDEVICE. */
int pmf_create(const pmf_options *opt, void *stream, void *workspace, size_t ws_bytes,
               pmf_handle **out);

/* Solve every lambda of n_inst instances (Sec. 2.1 schedule), packed into
 * shared launches.  flows_out (device, int64 [sum of L_i]) receives F in
 * (instance, lambda) order; status_out (device, int32 [n_inst], may be NULL)
 * receives PMF_OK, PMF_EINVAL / PMF_EOVERFLOW (bad capacities found on the
 * device; that instance's flows are -1) or PMF_ETIMEOUT (budget exhausted;
 * flows of unfinished lambdas are -1).  Masks stay in library memory until
 * the next solve or destroy (read them with pmf_extract_cut).
 * The call enqueues work on the handle's stream and returns when every
 * instance has finished; results are then complete in device memory.
 * Host-side errors (returned before any launch): PMF_EINVAL (K not 4 or 8,
 * W, H, L < 1, NULL pointers), PMF_ENOMEM, PMF_EDEVICE. */
int pmf_solve_batch(pmf_handle *h, const pmf_instance *inst, int32_t n_inst, int64_t *flows_out,
                    int32_t *status_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * pmf_solve_batch with every byte of solver state in a fixed device array of
 * PMF_NOALLOC_BYTES that the library holds on each device it runs on until
 * the process ends.  Arguments, results and errors are those of
 * pmf_solve_batch, and so are the flows and masks; the call itself allocates
 * no device memory (it launches supersteps directly, without capturing a
 * graph).  A batch whose state does not fit returns PMF_ELIMIT before any
 * launch; options.timing must be 0 (else PMF_EINVAL).  Masks stay readable
 * with pmf_extract_cut / pmf_extract_levels until the next solve on this
 * handle or the next no-allocation solve on this device: every handle on a
 * device shares the one array, so no-allocation solves on one device must
 * not overlap (they race on it). */
#define PMF_NOALLOC_BYTES ((size_t)64 << 20)
int pmf_solve_batch_noalloc(pmf_handle *h, const pmf_instance *inst, int32_t n_inst, int64_t *flows_out,
                            int32_t *status_out);

/* pmf_solve_batch that returns once the solve is set up: the superstep loop
 * (launches on the handle's stream and the host polls between them) runs on a
 * thread of the library while the caller goes on.  Same arguments, results
 * and host-side errors as pmf_solve_batch; the instance array is copied, the
 * device arrays it points to must stay valid until pmf_wait returns.  The
 * caller enqueues nothing on the handle's stream meanwhile (work on other
 * streams is fine).  pmf_wait blocks until the solve is done and returns its
 * status (what pmf_solve_batch would have returned; PMF_OK when no solve is
 * outstanding); pmf_query_done sets *done to 1 once it is done, 0 before,
 * without blocking.  Every other call on the handle first waits for the
 * outstanding solve. */
int pmf_solve_batch_async(pmf_handle *h, const pmf_instance *inst, int32_t n_inst, int64_t *flows_out,
                          int32_t *status_out);
int pmf_wait(pmf_handle *h);
int pmf_query_done(pmf_handle *h, int32_t *done);

/* Copy the minimal source side S_min of (instance inst, lambda index
 * lambda_idx) of the last solve -- inst is the index in the batch, or a
 * session slot id -- into mask_out (device, uint8 [H][W]):
 * 1 = source side (foreground), 0 = sink side.  Enqueued on the handle's
 * stream.  Errors: PMF_ENOTSOLVED (no solve yet, or that instance did not
 * finish), PMF_ERANGE. */
int pmf_extract_cut(pmf_handle *h, int32_t inst, int32_t lambda_idx, uint8_t *mask_out);

/* The masks of every lambda of a finished instance as one byte per pixel
 * (device, uint8 [H][W], caller-owned): the number of lambdas whose minimal
 * source side contains the pixel.  Because these sets are nested (they shrink
 * as lambda grows, Sec. 2.1), the mask of lambda index k is levels > k.
 * Enqueued on the handle's stream.  Errors: PMF_ENOTSOLVED (not finished),
 * PMF_ERANGE (bad id, or more than 255 lambdas). */
int pmf_extract_levels(pmf_handle *h, int32_t inst, uint8_t *levels_out);

/* Synchronise the stream and free everything the library allocated. */
int pmf_destroy(pmf_handle *h);

/* Static description of a status code. */
const char *pmf_strerror(int code);

/* Device bytes a solve of these instances needs (for admission by free
 * memory).  opt may be NULL. */
int pmf_query_bytes(const pmf_instance *inst, int32_t n_inst, const pmf_options *opt,
                    size_t *bytes);

/* ---- Serving: a resident session that instances join and leave ---------
 * Instance state stays in device memory between calls.  Requests are admitted
 * while earlier ones are still being solved and join the same launches at the
 * next superstep (continuous batching); every instance's result is the same
 * as when it is solved alone.  A handle is either in a session or used with
 * pmf_solve_batch (which opens a fresh session sized for its batch). */

typedef struct pmf_session_info {
    int64_t free_bytes;    /* free pool bytes                        */
    int64_t largest_free;  /* largest admissible instance block      */
    int32_t free_slots;    /* instance slots not in use              */
    int32_t admitted;      /* slots in use (running or finished)     */
    int32_t running;       /* admitted instances not yet finished    */
    int32_t reserved;
} pmf_session_info;

/* (Re)open the handle as a session with max_slots instance slots and a pool of
 * pool_bytes device bytes for instance state.  pool_bytes = 0 takes the whole
 * workspace, else opt->mem_budget, else half of the free device memory.
 * Discards earlier results.  Errors: PMF_EINVAL, PMF_ENOMEM, PMF_EDEVICE. */
int pmf_session_open(pmf_handle *h, int32_t max_slots, size_t pool_bytes);

/* Admit n_inst instances, all or none.  flows_out / status_out are as in
 * pmf_solve_batch (device memory owned by the caller; written when each
 * instance finishes).  ids_out (host int32 [n_inst], may be NULL) receives
 * the slot ids used by pmf_extract_cut and pmf_session_release.  Returns
 * PMF_EBUSY, admitting nothing, when slots or pool memory are short (the
 * caller retries after releasing finished instances). */
int pmf_session_submit(pmf_handle *h, const pmf_instance *inst, int32_t n_inst, int64_t *flows_out,
                       int32_t *status_out, int32_t *ids_out);

/* Run `supersteps` supersteps (1..65536) over every admitted, unfinished
 * instance, wait for them, and report the ids of the instances that finished
 * during this call in done_ids (host, room for max_ids; *n_done = how many
 * finished, which may exceed max_ids).  Their flows, status and masks are then
 * complete in device memory. */
int pmf_session_step(pmf_handle *h, int32_t supersteps, int32_t *done_ids, int32_t max_ids,
                     int32_t *n_done);

/* Return instance `id`'s slot and pool memory (an unfinished instance is
 * cancelled).  Its masks can no longer be read.  Errors: PMF_ERANGE. */
int pmf_session_release(pmf_handle *h, int32_t id);

/* Pool and slot occupancy, for admission by free memory. */
int pmf_session_query(pmf_handle *h, pmf_session_info *out);

/* The host-side checks pmf_solve_batch makes before any launch (K is 4 or 8;
 * W, H, L >= 1; W * H <= 2^29; nlink, cap_src, cap_snk0, lambdas non-NULL).
 * Reads no device memory, so it needs no GPU.  On failure *first_bad (may be
 * NULL) receives the index of the first offending instance.  Returns PMF_OK
 * or PMF_EINVAL. */
int pmf_check_instances(const pmf_instance *inst, int32_t n_inst, int32_t *first_bad);

/* Per device instance (slot) counters of the last solve or session, for
 * tuning and diagnosis: out (host, int64 [max_slots][8]) receives, for every
 * slot below max_slots, { finished (0/1), supersteps, sweep supersteps,
 * completed global relabels, relaxation passes, lambdas done, pixels swept,
 * pixels relaxed }.  In a pmf_solve_batch the chunks of caller instance i are
 * consecutive slots in caller order.  *n_slots = slots in use. */
int pmf_slot_stats(pmf_handle *h, int64_t *out, int32_t max_slots, int32_t *n_slots);

/* All breakpoints of one instance over an integer lambda range (paper
 * Sec. 2.1: the minimal source sets are nested as lambda grows and F is
 * concave and piecewise linear in lambda).  Finds every integer lambda c in
 * (lam_lo, lam_hi] with S_min(c) != S_min(c - 1), exactly: intervals whose end
 * sets differ in size are probed on both sides of the point where the two end
 * pieces of F meet and at points spread over the interval (up to 64 probes a
 * round, fewer for images too large for 64 solves in 1 GiB), and all probes
 * of a round are solved in one batched call on this handle.
 * inst->lambdas and inst->L are ignored; the other fields are as for
 * pmf_solve_batch (device pointers).  Blocking.
 *   bp_out   host, max_bp entries: the change points in increasing order
 *   f_out    host, max_bp + 1 entries or NULL: F(lam_lo), then F at each
 *            change point
 *   n_bp     the number of change points (even when larger than max_bp)
 *   exit_out device, W*H int32 or NULL: per pixel (row-major) the first lambda
 *            in [lam_lo, lam_hi] at which it is not in S_min (lam_lo if never
 *            in it, lam_hi + 1 if it never leaves)
 * Returns PMF_OK, PMF_ERANGE when more than max_bp change points exist (the
 * first max_bp are written), an instance status (PMF_EINVAL, PMF_EOVERFLOW,
 * PMF_ETIMEOUT) or PMF_ENOMEM / PMF_EDEVICE.  Replaces the handle's last
 * solve, also when it fails. */
int pmf_parametric(pmf_handle *h, const pmf_instance *inst, int32_t lam_lo, int32_t lam_hi, int32_t *bp_out,
                   int64_t *f_out, int32_t max_bp, int32_t *n_bp, int32_t *exit_out);

/* Every real breakpoint of one instance over [lam_lo, lam_hi] (paper
 * Sec. 2.1: F is the lower envelope of the lines c(S) + w(S) * lambda of the
 * source sets S, concave and piecewise linear, and the minimal source sets are
 * nested as lambda grows), exactly, as fractions: the lambdas x in
 * (lam_lo, lam_hi] at which S_min changes, i.e. the kinks of F.  The integer
 * search of pmf_parametric first finds each unit interval (c - 1, c] that
 * holds a change; the problem is then contracted to the pixels that change
 * inside it (those of S_min(c) joined to the source, those outside
 * S_min(c - 1) to the sink, as in the parametric algorithm of Gallo,
 * Grigoriadis and Tarjan), and each pair of known lines is probed where they
 * meet, x = p / q, by solving the contracted problem with every capacity
 * multiplied by q at lambda = p: F(x) on both lines confirms a breakpoint,
 * otherwise S_min(x) gives a new line between them.  All probes of a round are
 * solved in one batched call on this handle.  inst->lambdas and inst->L are
 * ignored; the other fields are as for pmf_solve_batch (device pointers).
 * Blocking.
 *   bp_num, bp_den  host, max_bp entries each: breakpoint j is
 *            bp_num[j] / bp_den[j] (lowest terms), increasing
 *   piece_a, piece_w  host, max_bp + 1 entries each: on piece j (from
 *            breakpoint j - 1, or lam_lo, to breakpoint j, or lam_hi),
 *            F(lambda) = piece_a[j] + piece_w[j] * lambda; piece_w[j] is the
 *            sink-slope sum of the free pixels of that piece's minimal set
 *   n_bp     the number of breakpoints (even when larger than max_bp)
 *   exit_out device, W*H int32, required: per pixel (row-major) the index
 *            of the first piece whose minimal set lacks it (0 if never in
 *            S_min, n_bp + 1 if it never leaves); also the working map of
 *            the search, so undefined after an error
 * Returns PMF_OK, PMF_ERANGE when more than max_bp breakpoints exist (the
 * first max_bp are written) or when a probe's scaled capacities would leave
 * the solver's int32 limits (q * capacity above PMF_INF or PMF_NLINK_MAX(K)),
 * an instance status (PMF_EINVAL, PMF_EOVERFLOW, PMF_ETIMEOUT) or PMF_ENOMEM
 * / PMF_EDEVICE.  Replaces the handle's last solve, also when it fails.
 * Device memory: that of pmf_parametric, then (K + 5) * 4 bytes per pixel of
 * the bounding box of each unit interval's changing pixels, kept for the
 * whole refinement, plus one round of up to 64 scaled probes of the largest
 * box and their solve. */
int pmf_breakpoints(pmf_handle *h, const pmf_instance *inst, int32_t lam_lo, int32_t lam_hi, int64_t *bp_num,
                    int64_t *bp_den, int64_t *piece_a, int64_t *piece_w, int32_t max_bp, int32_t *n_bp,
                    int32_t *exit_out);

/* Counters of the last solve. */
int pmf_get_stats(pmf_handle *h, pmf_stats *out);

/* Superstep trace of the last solve or session run with options.timing > 0
 * (empty otherwise): one row of PMF_TRACE_COLS int64 per superstep, { tiles
 * swept (4-connected instances), tiles swept (8-connected), tiles passed by
 * the relabel / cut / init passes (4-connected), the same (8-connected),
 * sweep ns and pass ns (timing = 2, else 0), control kernel ns, tile-work
 * ns }.
 * Copies min(rows, max_rows) rows to out (host) and returns the number of
 * rows recorded, or -PMF_EINVAL for a null handle, negative max_rows, or a
 * null out with max_rows > 0. */
#define PMF_TRACE_COLS 8
int64_t pmf_get_trace(pmf_handle *h, int64_t *out, int64_t max_rows);

#ifdef __cplusplus
}
#endif

#endif /* PMF_H */
