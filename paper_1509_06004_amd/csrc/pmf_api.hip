// Host side of libpmf: argument validation, device memory (a pool of
// per-instance blocks), the tile work list that packs all admitted instances
// into shared launches, and the superstep loop (direct launches or hipGraph
// replay).  pmf_solve_batch is a session that admits a whole batch at once
// and runs it to completion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "pmf.h"
#include "pmf_internal.h"
#include "pmf_parametric.h"

using namespace pmf;

namespace {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

void tile_dims(const pmf_options &o, int *tw, int *th) {
    *tw = o.tile_w == 64 ? 64 : 32;
    *th = 1024 / *tw;
}

bool valid_options(const pmf_options &o) {
    if (o.tile_w != 0 && o.tile_w != 32 && o.tile_w != 64) return false;
    if (o.tile_h != 0 && o.tile_w != 0 && o.tile_w * o.tile_h != 1024) return false;
    if (o.inner_iters < 1 || o.inner_iters > 4096) return false;
    if (o.sweeps_per_relabel < 1 || o.sweeps_per_relabel > 1 << 20) return false;
    if (o.local_bfs_iters < 1 || o.local_bfs_iters > 1 << 20) return false;
    if (o.exchange_rounds < 1 || o.exchange_rounds > 64) return false;
    if (o.tail_tiles < 0 || o.relabel_passes < 0) return false;
    if (o.orientation < kOrientAsGiven || o.orientation > kOrientExchange) return false;
    if (o.gap != 0 && o.gap != 1) return false;
    if (o.persist_tiles < 0 || o.persist_wgs < 0) return false;
    if (o.tail_sweep_exchanges < 0 || o.tail_sweep_exchanges > 64) return false;
    if (o.tail_tiles > 0 && (o.tail_inner_iters < 1 || o.tail_inner_iters > 4096 ||
                             o.tail_exchange_rounds < 1 || o.tail_exchange_rounds > 64))
        return false;
    if (o.steps_per_sync < 1 || o.steps_per_sync > 1 << 16) return false;
    if (o.max_supersteps < 1) return false;
    if (o.order != 0 && o.order != 1) return false;
    if (o.timing < 0 || o.timing > 2) return false;
    if (o.mem_budget < 0 || o.max_slots < 0) return false;
    return true;
}

int check_instance(const pmf_instance &I) {
    if (I.K != 4 && I.K != 8) return PMF_EINVAL;
    if (I.W < 1 || I.H < 1 || I.L < 1) return PMF_EINVAL;
    if ((int64_t)I.W * I.H > (int64_t)(1 << 29)) return PMF_EINVAL;  // heights and indices stay int32
    if (!I.nlink || !I.cap_src || !I.cap_snk0 || !I.lambdas) return PMF_EINVAL;
    return PMF_OK;
}

// Byte offsets of one instance's planes inside its block.
struct BlockLayout {
    size_t r, e, rt, h, inbox, rmask, masks, tile_act, tile_chg, tile_cnt, hist, total;
    int tiles_x, tiles_y;
};

BlockLayout block_layout(const pmf_instance &I, int tw, int th, bool gap) {
    BlockLayout b;
    b.tiles_x = (I.W + tw - 1) / tw;
    b.tiles_y = (I.H + th - 1) / th;
    const size_t px = (size_t)I.W * I.H, K = (size_t)I.K, nt = (size_t)b.tiles_x * b.tiles_y;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    b.r = take(4 * K * px);
    b.e = take(4 * px);
    b.rt = take(4 * px);
    b.h = take(4 * px);
    b.inbox = take(4 * nt * (size_t)border_words(I.K, tw, th));
    b.rmask = take(2 * px);
    b.masks = take((size_t)I.L * px);
    b.tile_act = take(4 * nt);
    b.tile_chg = take(2 * nt);
    b.tile_cnt = take(4 * nt);
    b.hist = gap ? take(4 * nt * (size_t)(tw * th)) : 0;
    b.total = off;
    return b;
}

// Work-list capacity for a pool: every tile's share of its instance block is
// at least 512 bytes, so the pool can never hold more tiles than this.
size_t worklist_cap(int slots, size_t pool_bytes) { return pool_bytes / 512 + (size_t)slots; }

// Device bytes of the control area for `slots` slots and a work list of `wl` tiles.
size_t control_bytes(int slots, size_t wl) {
    return align_up(sizeof(InstDesc) * (size_t)slots) + align_up(sizeof(InstState) * (size_t)slots) +
           align_up(4 * (size_t)slots) + align_up(256) + align_up(4 * (size_t)slots) + align_up(4 * 8 * wl) +
           align_up(sizeof(StepParams));
}

// First-fit allocator over [0, cap) with coalescing of freed ranges.
class Pool {
   public:
    void reset(size_t cap) {
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t sz, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= sz) {
                *off = it->first;
                const size_t rest = it->second - sz;
                const size_t at = it->first + sz;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t sz) {
        auto it = free_.emplace(off, sz).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const {
        size_t s = 0;
        for (auto &kv : free_) s += kv.second;
        return s;
    }
    size_t largest() const {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

   private:
    std::map<size_t, size_t> free_;
};

// The fixed device array of the no-allocation solves: every device the
// library runs on holds one until the process ends, shared by every handle
// on that device.  Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[PMF_NOALLOC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
char *scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per
// device, with that device current); null on failure.
char *scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        scratch_ptr[dev] = (char *)p;
    }
    return scratch_ptr[dev];
}

struct Slot {
    bool live = false;      // admitted and not released
    bool finished = false;  // completion seen by the host
    int32_t W = 0, H = 0, K = 0, L = 0, ntiles = 0, done_k = 0;
    int64_t work = 0;       // pixels x lambdas (packing order)
    size_t off = 0, bytes = 0;
    size_t masks = 0;       // arena offset of the masks
};

}  // namespace

struct pmf_handle {
    pmf_options opt;
    int tw = 32, th = 32;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    int device = 0;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    bool own_arena = true;
    int32_t *pinned = nullptr;  // host-visible copy of the counter block (completions, list sizes, barrier)
    int32_t *pinned_ring = nullptr;
    InstState *pinned_state = nullptr;
    // session
    bool open = false;
    int max_slots = 0;
    size_t wl_cap = 0;
    size_t pool_base = 0;
    Pool pool;
    std::vector<Slot> slots;
    std::vector<int> free_slots;  // stack, lowest id on top
    int32_t ring_seen = 0;
    bool wl_dirty = true;
    int64_t wl_finished = 0;  // finished instances still in the work list
    int64_t epoch_steps = 0;  // steps run since the work list last changed
    StepParams P;
    hipGraphExec_t graph = nullptr;
    int graph_S = 0;
    StepParams graph_P;  // the parameters the graph was captured with (a new work list of the same
                         // shape and place, e.g. the next batch of the same sizes, replays it as it is)
    pmf_stats stats;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // bracket every launch group (device time)
    // timing mode: six events per superstep of a host round (start and end
    // of the tile-work or sweep kernels, of the pass kernels, of the control
    // kernel) and a device buffer for the list sizes of each of those supersteps
    std::vector<hipEvent_t> kev;
    int32_t *trace_lists = nullptr;
    int trace_cap = 0;
    int64_t *kpx = nullptr;  // timing mode: pixel visits by kind, [0..7] tile-work launches, [8..15] persistent
    std::vector<int64_t> trace;  // timing mode: PMF_TRACE_COLS values per superstep
    // pmf_solve_batch: caller instance i = slots [user_first[i], user_first[i+1]),
    // lambda k of it in slot user_first[i] + k / chunk at index k % chunk
    bool batch = false;
    int32_t chunk = 1;
    // persistent supersteps: workgroups of the cooperative launch (0: not
    // available), tiles listed by the last superstep (-1: not known yet), and
    // whether a barrier wait gave up (the device state is then unusable)
    int persist_grid[3] = {0, 0, 0};  // by work-list connectivity: 4 only, 8 only, mixed
    size_t reserve_tail = 0;  // bytes at the end of the arena that sessions leave alone (pmf_parametric)
    // pmf_solve_batch_async: the thread running the superstep loop, the
    // instances it works on (a copy of the caller's array) and its status
    std::thread worker;
    std::vector<pmf_instance> async_inst;
    std::atomic<int> async_done{1};
    int async_rc = PMF_OK;
    int64_t last_listed = -1;
    bool poisoned = false;
    StepParams *P_dev = nullptr;          // device copy of P read by the persistent launch
    StepParams *pinned_params = nullptr;  // its staging copy
    // device memory the current session is laid out in: the arena, or memory
    // handed in for one solve (then polled through host vectors instead of
    // the pinned buffers, so that the solve allocates nothing)
    char *base = nullptr;
    bool ext = false;
    char *scratch_dev = nullptr;
    std::vector<int32_t> host_ring;
    std::vector<InstState> host_state;
    std::vector<int32_t> user_first, user_L;
};

namespace {

void drop_graph(pmf_handle *h) {
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
}

// Wait for an outstanding pmf_solve_batch_async (every call on a handle
// does, so the worker thread and the caller never use the handle together);
// returns that solve's status.
int finish_async(pmf_handle *h) {
    if (h->worker.joinable()) h->worker.join();
    const int rc = h->async_rc;
    h->async_rc = PMF_OK;
    return rc;
}

int ensure_arena(pmf_handle *h, size_t need) {
    if (need <= h->arena_bytes) return PMF_OK;
    if (!h->own_arena) return PMF_ENOMEM;
    if (h->opt.mem_budget > 0 && (int64_t)need > h->opt.mem_budget) return PMF_ENOMEM;
    if (h->arena) {
        // the last solve's or session's state lived there: it is gone
        (void)hipStreamSynchronize(h->stream);
        h->open = false;
        (void)hipFree(h->arena);
        h->arena = nullptr;
        h->arena_bytes = 0;
    }
    size_t want = need + need / 8;  // slack so that nearby sizes reuse the arena
    if (h->opt.mem_budget > 0 && (int64_t)want > h->opt.mem_budget) want = need;
    if (hipMalloc((void **)&h->arena, want) != hipSuccess) {
        (void)hipGetLastError();
        h->arena = nullptr;
        return PMF_ENOMEM;
    }
    h->arena_bytes = want;
    return PMF_OK;
}

// Lay out the control area at the start of the arena and the pool after it
// (or at the start of `ext_base`, ext_bytes of device memory handed in for
// one solve, which must hold both: PMF_ENOMEM otherwise; host buffers for
// polling are then ordinary host memory).
int open_session(pmf_handle *h, int slots, size_t pool_bytes, char *ext_base = nullptr, size_t ext_bytes = 0) {
    if (slots < 1) return PMF_EINVAL;
    h->open = false;  // a captured graph stays: it is replayed only while the parameters match
    (void)hipStreamSynchronize(h->stream);
    const size_t wl = worklist_cap(slots, pool_bytes);
    const size_t ctl = control_bytes(slots, wl);
    h->ext = ext_base != nullptr;
    size_t base_bytes = 0;
    if (h->ext) {
        if (ctl + pool_bytes > ext_bytes) return PMF_ENOMEM;
        h->base = ext_base;
        base_bytes = ext_bytes;
        h->host_ring.resize(slots);
        h->host_state.resize(slots);
    } else {
        int rc = ensure_arena(h, ctl + pool_bytes + h->reserve_tail);
        if (rc != PMF_OK) return rc;
        h->base = h->arena;
        base_bytes = h->arena_bytes - h->reserve_tail;
    }
    if (!h->ext && ((int)h->slots.size() < slots || !h->pinned_ring)) {
        if (h->pinned_state) (void)hipHostFree(h->pinned_state);
        if (h->pinned_ring) (void)hipHostFree(h->pinned_ring);
        h->pinned_state = nullptr;
        h->pinned_ring = nullptr;
        if (hipHostMalloc((void **)&h->pinned_ring, 4 * (size_t)slots, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&h->pinned_state, sizeof(InstState) * (size_t)slots, hipHostMallocDefault) !=
                hipSuccess) {
            (void)hipGetLastError();
            return PMF_ENOMEM;
        }
    }
    char *A = h->base;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += align_up(bytes);
        return A + at;
    };
    StepParams &P = h->P;
    std::memset(&P, 0, sizeof(P));
    P.desc = (InstDesc *)take(sizeof(InstDesc) * (size_t)slots);
    P.st = (InstState *)take(sizeof(InstState) * (size_t)slots);
    P.ring = (int32_t *)take(4 * (size_t)slots);
    P.ring_count = (int32_t *)take(256);
    P.wl_slot = (const int32_t *)take(4 * (size_t)slots);
    P.lists = (int32_t *)take(4 * 8 * wl);
    h->P_dev = (StepParams *)take(sizeof(StepParams));
    P.list_count = P.ring_count + 4;  // counter block: [0] ring, [4..11] lists
    P.list_cap = (int32_t)wl;
    P.ring_cap = slots;
    P.nslots = slots;
    P.inner_iters = h->opt.inner_iters;
    P.sweeps_per_relabel = h->opt.sweeps_per_relabel;
    P.local_bfs_iters = h->opt.local_bfs_iters;
    P.exchange_rounds = h->opt.exchange_rounds;
    P.tail_tiles = h->opt.tail_tiles;
    P.tail_inner_iters = h->opt.tail_inner_iters;
    P.tail_exchange_rounds = h->opt.tail_exchange_rounds;
    P.tail_sweep_exchanges = h->opt.tail_sweep_exchanges;
    P.relabel_passes = h->opt.relabel_passes;
    P.orientation = h->opt.orientation;
    P.gap = h->opt.gap;
    P.max_steps = h->opt.max_supersteps;
    h->pool_base = off;
    // the work list is sized for pool_bytes, so the pool must not exceed it
    h->pool.reset(std::min(base_bytes - off, pool_bytes));
    h->max_slots = slots;
    h->wl_cap = wl;
    h->slots.assign(slots, Slot());
    h->free_slots.clear();
    for (int i = slots - 1; i >= 0; --i) h->free_slots.push_back(i);
    h->ring_seen = 0;
    h->wl_dirty = true;
    h->epoch_steps = 0;
    h->last_listed = -1;
    h->poisoned = false;
    if (h->kpx && hipMemsetAsync(h->kpx, 0, 16 * sizeof(int64_t), h->stream) != hipSuccess) return PMF_EDEVICE;
    std::memset(&h->stats, 0, sizeof(h->stats));
    h->trace.clear();
    h->stats.device_bytes = (int64_t)base_bytes;
    // every slot starts idle; the completion counter at zero
    if (hipMemsetAsync(P.st, 0, sizeof(InstState) * (size_t)slots, h->stream) != hipSuccess ||
        hipMemsetAsync(P.ring_count, 0, 256, h->stream) != hipSuccess)
        return PMF_EDEVICE;
    h->open = true;
    return PMF_OK;
}

// Rebuild the work list: every tile of every admitted, unfinished instance,
// 4-connected instances first, each group in FIFO or LPT (largest first)
// order (the "largest processing time first" rule of Sec. 3.3.1).
int rebuild_worklist(pmf_handle *h) {
    std::vector<int> ids;
    for (int i = 0; i < h->max_slots; ++i)
        if (h->slots[i].live && !h->slots[i].finished) ids.push_back(i);
    const bool lpt = h->opt.order == 1;
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
        const Slot &x = h->slots[a], &y = h->slots[b];
        if (x.K != y.K) return x.K < y.K;
        return lpt ? x.work > y.work : false;
    });
    int64_t t4 = 0, t8 = 0;
    for (int i : ids) (h->slots[i].K == 4 ? t4 : t8) += h->slots[i].ntiles;
    if ((size_t)(t4 + t8) > h->wl_cap) return PMF_ENOMEM;
    StepParams &P = h->P;
    P.ntiles = (int32_t)(t4 + t8);
    P.t4_count = (int32_t)t4;
    P.t8_count = (int32_t)t8;
    P.nwl = (int32_t)ids.size();
    P.wl_ident = 1;
    for (size_t w = 0; w < ids.size(); ++w) P.wl_ident &= ids[w] == (int)w ? 1 : 0;
    if (!ids.empty()) {
        std::vector<int32_t> wl(ids.begin(), ids.end());
        if (hipMemcpyAsync((void *)P.wl_slot, wl.data(), 4 * wl.size(), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess)
            return PMF_EDEVICE;
        // pageable source: the copy must finish before the vector goes
        if (hipStreamSynchronize(h->stream) != hipSuccess) return PMF_EDEVICE;
    }
    h->wl_dirty = false;
    h->wl_finished = 0;
    h->epoch_steps = 0;
    return PMF_OK;
}

int submit(pmf_handle *h, const pmf_instance *inst, int n, int64_t *flows_out, int32_t *status_out,
           int32_t *ids_out, const uint8_t *check_prev = nullptr) {
    if (!h->open) return PMF_EINVAL;
    if (n < 0 || (n > 0 && (!inst || !flows_out))) return PMF_EINVAL;
    for (int i = 0; i < n; ++i) {
        const int rc = check_instance(inst[i]);
        if (rc != PMF_OK) return rc;
    }
    if ((size_t)n > h->free_slots.size()) return PMF_EBUSY;
    // all or nothing: allocate every block first
    std::vector<size_t> offs(n);
    std::vector<BlockLayout> lay(n);
    int got = 0;
    for (; got < n; ++got) {
        lay[got] = block_layout(inst[got], h->tw, h->th, h->opt.gap != 0);
        if (!h->pool.alloc(lay[got].total, &offs[got])) break;
    }
    if (got < n) {
        for (int i = 0; i < got; ++i) h->pool.release(offs[i], lay[i].total);
        return PMF_EBUSY;
    }
    std::vector<InstDesc> desc(n);
    std::vector<InstState> st(n);
    std::vector<int> ids(n);
    int64_t lam_base = 0;
    for (int i = 0; i < n; ++i) {
        const pmf_instance &I = inst[i];
        const BlockLayout &B = lay[i];
        char *base = h->base + h->pool_base + offs[i];
        const int id = h->free_slots.back();
        h->free_slots.pop_back();
        ids[i] = id;
        InstDesc &D = desc[i];
        std::memset(&D, 0, sizeof(D));
        D.W = I.W;
        D.H = I.H;
        D.K = I.K;
        D.n = I.W * I.H;
        D.tiles_x = B.tiles_x;
        D.tiles_y = B.tiles_y;
        D.ntiles = B.tiles_x * B.tiles_y;
        D.tile0 = 0;
        D.L = I.L;
        D.slot_id = id;
        D.check_prev = check_prev ? check_prev[i] : 0;
        D.tile_w = h->tw;
        D.lambdas = I.lambdas;
        D.nlink = I.nlink;
        D.cap_src = I.cap_src;
        D.cap_snk0 = I.cap_snk0;
        D.slope = I.snk_slope;
        D.seed = I.seed;
        D.r = (int32_t *)(base + B.r);
        D.e = (int32_t *)(base + B.e);
        D.rt = (int32_t *)(base + B.rt);
        D.h = (int32_t *)(base + B.h);
        D.inbox = (int32_t *)(base + B.inbox);
        D.rmask = (uint16_t *)(base + B.rmask);
        D.masks = (uint8_t *)(base + B.masks);
        D.tile_act = (uint32_t *)(base + B.tile_act);
        D.tile_chg = (uint8_t *)(base + B.tile_chg);
        D.tile_cnt = (int32_t *)(base + B.tile_cnt);
        D.hist = h->opt.gap ? (int32_t *)(base + B.hist) : nullptr;
        D.hsize = h->opt.gap ? D.ntiles * h->tw * h->th : 0;
        D.flows = flows_out + lam_base;
        D.status = status_out ? status_out + i : nullptr;
        lam_base += I.L;
        std::memset(&st[i], 0, sizeof(InstState));
        const int pol = h->opt.orientation;
        st[i].phase = (pol == kOrientMoreSink || pol == kOrientMoreSource) ? kOrient : kInit;
        st[i].swap = pol == kOrientExchange ? 1 : 0;
        st[i].gap = kHInf;
        Slot &s = h->slots[id];
        s = Slot();
        s.live = true;
        s.W = I.W;
        s.H = I.H;
        s.K = I.K;
        s.L = I.L;
        s.ntiles = D.ntiles;
        s.work = (int64_t)I.W * I.H * I.L;
        s.off = offs[i];
        s.bytes = B.total;
        s.masks = h->pool_base + offs[i] + B.masks;
        if (ids_out) ids_out[i] = id;
    }
    // descriptors and states go to their slots, one copy per run of
    // consecutive ids (ids need not be contiguous; a fresh batch is one run)
    for (int i = 0; i < n;) {
        int j = i + 1;
        while (j < n && ids[j] == ids[j - 1] + 1) ++j;
        const size_t cnt = (size_t)(j - i);
        if (hipMemcpyAsync(h->P.desc + ids[i], &desc[i], sizeof(InstDesc) * cnt, hipMemcpyHostToDevice,
                           h->stream) != hipSuccess ||
            hipMemcpyAsync(h->P.st + ids[i], &st[i], sizeof(InstState) * cnt, hipMemcpyHostToDevice, h->stream) !=
                hipSuccess)
            return PMF_EDEVICE;
        i = j;
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) return PMF_EDEVICE;
    if (n) h->wl_dirty = true;
    return PMF_OK;
}

// Timing mode: room for the events and list sizes of `steps` supersteps.
int ensure_timing(pmf_handle *h, int steps) {
    if (!h->kpx) {
        if (hipMalloc((void **)&h->kpx, 16 * sizeof(int64_t)) != hipSuccess) {
            (void)hipGetLastError();
            h->kpx = nullptr;
            return PMF_ENOMEM;
        }
        if (hipMemsetAsync(h->kpx, 0, 16 * sizeof(int64_t), h->stream) != hipSuccess) return PMF_EDEVICE;
    }
    while ((int)h->kev.size() < 6 * steps) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return PMF_EDEVICE;
        h->kev.push_back(e);
    }
    if (h->trace_cap < steps) {
        if (h->trace_lists) {
            (void)hipStreamSynchronize(h->stream);
            (void)hipFree(h->trace_lists);
            h->trace_lists = nullptr;
            h->trace_cap = 0;
        }
        if (hipMalloc((void **)&h->trace_lists, 16 * (size_t)steps) != hipSuccess) {
            (void)hipGetLastError();
            return PMF_ENOMEM;
        }
        h->trace_cap = steps;
    }
    return PMF_OK;
}

// Timing mode, after `steps` supersteps have completed: kernel times from the
// events and one trace row per superstep (its list sizes and the three times).
int read_kernel_events(pmf_handle *h, int steps) {
    std::vector<int32_t> cnt(4 * (size_t)steps);
    if (hipMemcpy(cnt.data(), h->trace_lists, 16 * (size_t)steps, hipMemcpyDeviceToHost) != hipSuccess)
        return PMF_EDEVICE;
    const bool split = h->opt.timing == 2;
    for (int i = 0; i < steps; ++i) {
        hipEvent_t *ev = h->kev.data() + 6 * i;
        float a = 0.f, b = 0.f, c = 0.f;
        if (hipEventElapsedTime(&a, ev[0], ev[1]) != hipSuccess) a = 0.f;
        if (split && hipEventElapsedTime(&b, ev[2], ev[3]) != hipSuccess) b = 0.f;
        if (hipEventElapsedTime(&c, ev[4], ev[5]) != hipSuccess) c = 0.f;
        const int64_t na = (int64_t)(a * 1e6), nb = (int64_t)(b * 1e6), nc = (int64_t)(c * 1e6);
        const int64_t sw = split ? na : 0, ps = split ? nb : 0, work = na + nb;
        h->stats.work_ns += work;
        h->stats.sweep_ns += sw;
        h->stats.pass_ns += ps;
        h->stats.control_ns += nc;
        const int32_t *c4 = cnt.data() + 4 * i;
        const int64_t row[PMF_TRACE_COLS] = {c4[0], c4[1], c4[2], c4[3], sw, ps, nc, work};
        h->trace.insert(h->trace.end(), row, row + PMF_TRACE_COLS);
    }
    return PMF_OK;
}

// Launch `steps` supersteps (or, in the latency-bound tail, one persistent
// launch of up to `persist_steps`), wait, and collect the slots that finished.
int run_steps(pmf_handle *h, int steps, std::vector<int> *finished, int persist_steps = 0) {
    if (h->poisoned) return PMF_EDEVICE;
    if (h->wl_dirty) {
        const int rc = rebuild_worklist(h);
        if (rc != PMF_OK) return rc;
    }
    StepParams &P = h->P;
    hipStream_t s = h->stream;
    const bool timing = h->opt.timing != 0;
    bool persisted = false;
    if (timing) {
        const int rc = ensure_timing(h, steps);
        if (rc != PMF_OK) return rc;
    }
    const int kset = P.t8_count == 0 ? 4 : P.t4_count == 0 ? 8 : 12;
    int &pgrid = h->persist_grid[kset == 4 ? 0 : kset == 8 ? 1 : 2];
    if (P.ntiles > 0 && h->opt.persist_tiles > 0 && !h->opt.gap && pgrid >= 8 && h->last_listed >= 0 &&
        h->last_listed < h->opt.persist_tiles) {
        const int budget = std::max(steps, persist_steps);
        if (hipEventRecord(h->ev0, s) != hipSuccess) return PMF_EDEVICE;
        const int exit_tiles = (int)std::min<int64_t>(2 * (int64_t)h->opt.persist_tiles, INT32_MAX);
        *h->pinned_params = P;
        if (timing) h->pinned_params->kpx = h->kpx + 8;
        if (hipMemcpyAsync(h->P_dev, h->pinned_params, sizeof(StepParams), hipMemcpyHostToDevice, s) != hipSuccess)
            return PMF_EDEVICE;
        if (launch_persist(h->P_dev, h->tw, kset, pgrid, budget, exit_tiles, s) == 0) {
            if (hipEventRecord(h->ev1, s) != hipSuccess) return PMF_EDEVICE;
            persisted = true;
            h->stats.persist_launches += 1;
        } else {
            pgrid = 0;  // refused (e.g. not co-resident): supersteps as separate launches
        }
    }
    if (P.ntiles > 0 && !persisted) {
        // replay a captured graph: a batch's work list from its first superstep
        // (it stays the same for the whole solve), a session's once it has been
        // used once; the graph is captured again when the parameters changed
        const bool use_graph = h->opt.use_graph && !timing && !h->ext && (h->batch || h->epoch_steps > 0);
        if (use_graph && (!h->graph || h->graph_S != steps || std::memcmp(&h->graph_P, &P, sizeof(P)) != 0)) {
            drop_graph(h);
            hipGraph_t g = nullptr;
            bool ok = hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
            for (int i = 0; ok && i < steps; ++i) ok = launch_superstep(P, h->tw, h->capture) >= 0;
            const bool ended = hipStreamEndCapture(h->capture, &g) == hipSuccess;
            ok = ok && ended && hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            if (!ok) {
                (void)hipGetLastError();
                drop_graph(h);
                return PMF_EDEVICE;
            }
            h->graph_S = steps;
            h->graph_P = P;
        }
        if (hipEventRecord(h->ev0, s) != hipSuccess) return PMF_EDEVICE;
        if (use_graph) {
            if (hipGraphLaunch(h->graph, s) != hipSuccess) return PMF_EDEVICE;
            h->stats.work_launches += (int64_t)steps * ((P.t4_count > 0) + (P.t8_count > 0));
        } else {
            for (int i = 0; i < steps; ++i) {
                StepParams Pi = P;
                if (timing) {
                    Pi.trace_lists = h->trace_lists + 4 * i;
                    Pi.kpx = h->kpx;
                }
                const int ns = launch_superstep(Pi, h->tw, s, timing ? (void *const *)(h->kev.data() + 6 * i) : nullptr,
                                                h->opt.timing == 2);
                if (ns < 0) return PMF_EDEVICE;
                h->stats.work_launches += ns;
            }
        }
        if (hipEventRecord(h->ev1, s) != hipSuccess) return PMF_EDEVICE;
        h->stats.supersteps += steps;
        h->epoch_steps += steps;
    }
    // A batch (few slots, all admitted at once) copies the whole completion
    // ring and every slot's state along with the completion count: one round
    // trip per sync instead of two and a copy per finished instance.
    const int cap = h->max_slots;
    const bool bulk = h->batch && !h->ext && (size_t)cap * sizeof(InstState) <= ((size_t)1 << 20);
    int32_t *ringb = h->ext ? h->host_ring.data() : h->pinned_ring;
    InstState *stateb = h->ext ? h->host_state.data() : h->pinned_state;
    // device-to-host copy of polled data: queued on the stream into pinned
    // memory, or (memory handed in: ordinary host memory) synchronous once
    // the stream is idle
    auto d2h = [&](void *dst, const void *src, size_t bytes) -> bool {
        if (h->ext) return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) == hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) == hipSuccess;
    };
    // the counter block: completions, list sizes of the last superstep, barrier words
    if (hipMemcpyAsync(h->pinned, P.ring_count, 4 * (kBarSteps + 1), hipMemcpyDeviceToHost, s) != hipSuccess)
        return PMF_EDEVICE;
    if (bulk && (!d2h(ringb, P.ring, 4 * (size_t)cap) || !d2h(stateb, P.st, sizeof(InstState) * (size_t)cap)))
        return PMF_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return PMF_EDEVICE;
    h->stats.host_syncs += 1;
    if (P.ntiles > 0) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) {
            h->stats.device_ns += (int64_t)(ms * 1e6);
            if (persisted) h->stats.persist_ns += (int64_t)(ms * 1e6);
        }
        if (timing && !persisted) {
            const int rc = read_kernel_events(h, steps);
            if (rc != PMF_OK) return rc;
        }
        if (timing && hipMemcpy(h->stats.kernel_px, h->kpx, 16 * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
            return PMF_EDEVICE;
    }
    const volatile int32_t *cb = h->pinned;
    if (persisted) {
        if (cb[kBarAbort] != 0) {
            h->poisoned = true;  // a superstep was left half done
            return PMF_EDEVICE;
        }
        const int ran = cb[kBarSteps];
        h->stats.supersteps += ran;
        h->stats.persist_supersteps += ran;
        h->epoch_steps += ran;
    }
    if (P.ntiles > 0) h->last_listed = (int64_t)cb[8] + cb[9] + cb[10] + cb[11];
    const int32_t count = cb[0];
    if (count <= h->ring_seen) return PMF_OK;
    // the new ring entries (at most two contiguous ranges), then the final
    // states of those instances (one bulk copy when many finished)
    const int32_t fresh = count - h->ring_seen;
    if (fresh > cap) return PMF_EDEVICE;  // a slot can finish only once per admission
    if (!bulk) {
        const int a0 = h->ring_seen % cap;
        const int first_len = std::min(fresh, cap - a0);
        if (!d2h(ringb + a0, P.ring + a0, 4 * (size_t)first_len)) return PMF_EDEVICE;
        if (fresh > first_len && !d2h(ringb, P.ring, 4 * (size_t)(fresh - first_len))) return PMF_EDEVICE;
        if (hipStreamSynchronize(s) != hipSuccess) return PMF_EDEVICE;
    }
    std::vector<int> got;
    for (int32_t c = h->ring_seen; c < count; ++c) {
        const int id = ringb[c % cap];
        if (id < 0 || id >= cap) return PMF_EDEVICE;
        got.push_back(id);
    }
    if (!bulk) {
        if (got.size() > 64) {
            if (!d2h(stateb, P.st, sizeof(InstState) * (size_t)cap)) return PMF_EDEVICE;
        } else {
            for (int id : got)
                if (!d2h(stateb + id, P.st + id, sizeof(InstState))) return PMF_EDEVICE;
        }
        if (hipStreamSynchronize(s) != hipSuccess) return PMF_EDEVICE;
    }
    h->ring_seen = count;
    for (int id : got) {
        Slot &sl = h->slots[id];
        const InstState &x = stateb[id];
        sl.finished = true;
        sl.done_k = x.k;
        h->stats.px_init += x.px_init;
        h->stats.px_sweep += x.px_sweep;
        h->stats.px_relabel += x.px_relabel;
        h->stats.px_cut += x.px_cut;
        h->stats.px_orient += x.px_orient;
        h->stats.px_init_x += x.px_init_x;
        h->stats.px_cut_x += x.px_cut_x;
        h->stats.gap_kills += x.gap_kills;
        h->stats.sweep_visits += x.sweeps;
        h->stats.global_relabels += x.relabels;
        h->stats.bfs_passes += x.passes;
        if (finished) finished->push_back(id);
    }
    // Finished instances stay in the work list (their compaction and control
    // return at once), so a completion alone neither rebuilds the list nor
    // drops the captured graph; the list is rebuilt once they are half of it
    // (and whenever instances are admitted or cancelled).
    h->wl_finished += (int64_t)got.size();
    if (2 * h->wl_finished > (int64_t)P.nwl) h->wl_dirty = true;
    return PMF_OK;
}

}  // namespace

extern "C" {

void pmf_default_options(pmf_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tile_w = 32;
    o->tile_h = 32;
    o->inner_iters = 12;
    o->sweeps_per_relabel = 12;
    o->local_bfs_iters = 16;
    o->exchange_rounds = 2;
    o->tail_tiles = 2048;
    o->tail_inner_iters = 32;
    o->tail_exchange_rounds = 16;
    o->orientation = kOrientMoreSource;
    o->steps_per_sync = 32;
    o->max_supersteps = 2000000;
    o->use_graph = 1;
    o->order = 1;
    o->mem_budget = 0;
    o->max_slots = 4096;
}

const char *pmf_strerror(int code) {
    switch (code) {
        case PMF_OK: return "ok";
        case PMF_EINVAL: return "invalid argument or capacity value";
        case PMF_EOVERFLOW: return "capacities exceed the int32 headroom";
        case PMF_ENOMEM: return "not enough device memory or workspace";
        case PMF_EDEVICE: return "HIP runtime error";
        case PMF_ETIMEOUT: return "superstep budget exhausted";
        case PMF_ENOTSOLVED: return "no completed solve for this instance and lambda";
        case PMF_ERANGE: return "instance or lambda index out of range";
        case PMF_EBUSY: return "no free slot or pool memory";
        case PMF_ELIMIT: return "batch does not fit the fixed buffer of pmf_solve_batch_noalloc";
        default: return "unknown status";
    }
}

int pmf_create(const pmf_options *opt, void *stream, void *workspace, size_t ws_bytes, pmf_handle **out) {
    if (!out) return PMF_EINVAL;
    *out = nullptr;
    pmf_options o;
    if (opt)
        o = *opt;
    else
        pmf_default_options(&o);
    if (o.tile_w == 0) o.tile_w = 32;
    if (o.tile_h == 0) o.tile_h = 1024 / o.tile_w;
    if (o.max_slots == 0) o.max_slots = 4096;
    if (o.exchange_rounds == 0) o.exchange_rounds = 1;
    if (!valid_options(o)) return PMF_EINVAL;
    if (workspace && ws_bytes == 0) return PMF_EINVAL;
    pmf_handle *h = new (std::nothrow) pmf_handle();
    if (!h) return PMF_ENOMEM;
    h->opt = o;
    tile_dims(o, &h->tw, &h->th);
    h->stream = (hipStream_t)stream;
    std::memset(&h->stats, 0, sizeof(h->stats));
    std::memset(&h->P, 0, sizeof(h->P));
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return PMF_EDEVICE;
    }
    if (workspace) {
        h->arena = (char *)workspace;
        h->arena_bytes = ws_bytes;
        h->own_arena = false;
    }
    if (hipHostMalloc((void **)&h->pinned, 256, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&h->pinned_params, sizeof(StepParams), hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
        (void)hipGetLastError();
        pmf_destroy(h);
        return PMF_EDEVICE;
    }
    h->scratch_dev = scratch_address(h->device);
    if (o.persist_tiles > 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) cus = 0;
        const int want = o.persist_wgs > 0 ? o.persist_wgs : cus;
        const int ksets[3] = {4, 8, 12};
        for (int i = 0; i < 3; ++i)
            h->persist_grid[i] = (std::min(want, persist_workgroups(h->tw, ksets[i])) / 8) * 8;
    }
    *out = h;
    return PMF_OK;
}

int pmf_check_instances(const pmf_instance *inst, int32_t n_inst, int32_t *first_bad) {
    if (first_bad) *first_bad = -1;
    if (n_inst < 0 || (n_inst > 0 && !inst)) return PMF_EINVAL;
    for (int i = 0; i < n_inst; ++i) {
        if (check_instance(inst[i]) != PMF_OK) {
            if (first_bad) *first_bad = i;
            return PMF_EINVAL;
        }
    }
    return PMF_OK;
}

int pmf_query_bytes(const pmf_instance *inst, int32_t n, const pmf_options *opt, size_t *bytes) {
    if (!bytes || n < 0 || (n > 0 && !inst)) return PMF_EINVAL;
    pmf_options o;
    if (opt)
        o = *opt;
    else
        pmf_default_options(&o);
    int tw, th;
    tile_dims(o, &tw, &th);
    size_t pool = 0;
    for (int i = 0; i < n; ++i) {
        if (check_instance(inst[i]) != PMF_OK) return PMF_EINVAL;
        pool += block_layout(inst[i], tw, th, o.gap != 0).total;
    }
    *bytes = pool;
    return PMF_OK;
}

}  // extern "C"

namespace {

// Bytes of the pool for a batch whose schedules are cut into chunks of C lambdas.
size_t batch_pool_bytes(const pmf_instance *inst, int n, int C, int tw, int th, bool gap, int64_t *n_sub) {
    size_t pool = 0;
    int64_t subs = 0;
    for (int i = 0; i < n; ++i) {
        pmf_instance I = inst[i];
        const int full = I.L / C, rest = I.L % C;
        if (full) {
            I.L = C;
            pool += (size_t)full * block_layout(I, tw, th, gap).total;
        }
        if (rest) {
            I.L = rest;
            pool += block_layout(I, tw, th, gap).total;
        }
        subs += full + (rest ? 1 : 0);
    }
    pool += align_up(8 * (3 * (size_t)n + 1)) + align_up(4 * (size_t)subs);  // finalize metadata
    *n_sub = subs;
    return pool;
}

// The lambda chunk: the caller's choice, else chosen in two steps.  Chunks
// run concurrently and each lambda after the first of a chunk is warm-started
// from the one before, so short chunks give more parallel work (a shorter
// critical path of supersteps) and long ones less work in total.  First the
// smallest chunk whose state fits the memory available to the handle; then
// the longest chunk from there that still gives every workgroup the device
// holds at once kTilesPerWorkgroup tiles, counting the resident workgroups
// of the connectivity that holds most of the batch's tiles (measured on the
// 500x375 25-seed x 20-lambda batch: chunks of 2 lambdas at 4-connectivity
// and of 3-4 at 8 were fastest; the rule picks 2 and 3, -7% and -20% against
// chunks of 1).
constexpr int64_t kTilesPerWorkgroup = 40;

int64_t batch_tiles(const pmf_instance *inst, int n, int C, int tw, int th, int64_t *t8) {
    int64_t t = 0, e = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t tiles = (int64_t)((inst[i].W + tw - 1) / tw) * ((inst[i].H + th - 1) / th);
        const int64_t v = tiles * ((inst[i].L + C - 1) / C);
        t += v;
        if (inst[i].K == 8) e += v;
    }
    if (t8) *t8 = e;
    return t;
}

int longest_parallel_chunk(pmf_handle *h, const pmf_instance *inst, int n, int C, int maxL) {
    int64_t t8 = 0;
    const int64_t t = batch_tiles(inst, n, 1, h->tw, h->th, &t8);
    const int res = resident_workgroups(2 * t8 >= t ? 8 : 4, h->tw);
    if (res <= 0) return C;
    const int64_t target = kTilesPerWorkgroup * res;
    while (C < maxL && batch_tiles(inst, n, C + 1, h->tw, h->th, nullptr) >= target) ++C;
    return C;
}

int choose_chunk(pmf_handle *h, const pmf_instance *inst, int n, size_t ext_bytes) {
    int maxL = 1;
    for (int i = 0; i < n; ++i) maxL = std::max(maxL, (int)inst[i].L);
    if (h->opt.lambda_chunk > 0) return std::min((int)h->opt.lambda_chunk, maxL);
    size_t budget;
    if (ext_bytes) {
        budget = ext_bytes;
    } else if (!h->own_arena) {
        budget = h->arena_bytes;
    } else if (h->opt.mem_budget > 0) {
        budget = (size_t)h->opt.mem_budget;
    } else {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return maxL;
        budget = (size_t)((double)(fr + h->arena_bytes) * 0.7);
    }
    for (int C = 1;; C = C < 4 ? C + 1 : C * 2) {
        if (C >= maxL) return maxL;
        int64_t subs = 0;
        const size_t pool = batch_pool_bytes(inst, n, C, h->tw, h->th, h->opt.gap != 0, &subs);
        if (subs <= (1 << 20) && pool + control_bytes((int)subs, worklist_cap((int)subs, pool)) <= budget)
            return longest_parallel_chunk(h, inst, n, C, maxL);
    }
}

// Slot and lambda index inside it of (caller instance, lambda).
int locate(pmf_handle *h, int32_t inst, int32_t lambda_idx, int *slot, int *k) {
    if (h->batch) {
        if (inst < 0 || inst >= (int)h->user_L.size()) return PMF_ERANGE;
        if (lambda_idx < 0 || lambda_idx >= h->user_L[inst]) return PMF_ERANGE;
        *slot = h->user_first[inst] + lambda_idx / h->chunk;
        *k = lambda_idx % h->chunk;
        return PMF_OK;
    }
    if (inst < 0 || inst >= h->max_slots || !h->slots[inst].live) return PMF_ERANGE;
    if (lambda_idx < 0 || lambda_idx >= h->slots[inst].L) return PMF_ERANGE;
    *slot = inst;
    *k = lambda_idx;
    return PMF_OK;
}

// pmf_solve_batch, with its state in the arena or in ext_bytes of device
// memory at ext_base (a solve that allocates nothing).
int solve_batch(pmf_handle *h, const pmf_instance *inst, int32_t n_inst, int64_t *flows_out, int32_t *status_out,
                char *ext_base = nullptr, size_t ext_bytes = 0) {
    if (!h || n_inst < 0 || (n_inst > 0 && (!inst || !flows_out))) return PMF_EINVAL;
    int rc = pmf_check_instances(inst, n_inst, nullptr);
    if (rc != PMF_OK) return rc;
    const int C = n_inst ? choose_chunk(h, inst, n_inst, ext_base ? ext_bytes : 0) : 1;
    int64_t n_sub = 0;
    const size_t pool = batch_pool_bytes(inst, n_inst, C, h->tw, h->th, h->opt.gap != 0, &n_sub);
    rc = open_session(h, (int)std::max<int64_t>(n_sub, 1), pool, ext_base, ext_bytes);
    if (rc != PMF_OK) return rc;
    h->batch = true;
    h->chunk = C;
    h->user_first.assign(n_inst + 1, 0);
    h->user_L.assign(n_inst, 0);
    if (n_inst == 0) return PMF_OK;
    // chunks in caller order, so that their flows are contiguous in flows_out
    std::vector<pmf_instance> subs;
    std::vector<uint8_t> prev;
    std::vector<int64_t> meta(3 * (size_t)n_inst + 1);
    int64_t foff = 0;
    for (int i = 0; i < n_inst; ++i) {
        h->user_first[i] = (int32_t)subs.size();
        h->user_L[i] = inst[i].L;
        meta[i] = (int64_t)subs.size();
        meta[n_inst + 1 + i] = foff;
        meta[2 * n_inst + 1 + i] = inst[i].L;
        foff += inst[i].L;
        for (int a = 0; a < inst[i].L; a += C) {
            pmf_instance I = inst[i];
            I.lambdas = inst[i].lambdas + a;
            I.L = std::min(C, inst[i].L - a);
            subs.push_back(I);
            prev.push_back(a > 0 ? 1 : 0);
        }
    }
    meta[n_inst] = (int64_t)subs.size();
    h->user_first[n_inst] = (int32_t)subs.size();
    // the finalize metadata takes the first pool block
    size_t moff = 0;
    const size_t mbytes = align_up(8 * meta.size()) + align_up(4 * subs.size());
    if (!h->pool.alloc(mbytes, &moff)) return PMF_ENOMEM;
    char *mbase = h->base + h->pool_base + moff;
    int64_t *d_meta = (int64_t *)mbase;
    int32_t *d_sub_status = (int32_t *)(mbase + align_up(8 * meta.size()));
    if (hipMemcpyAsync(d_meta, meta.data(), 8 * meta.size(), hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return PMF_EDEVICE;
    rc = submit(h, subs.data(), (int)subs.size(), flows_out, d_sub_status, nullptr, prev.data());
    if (rc != PMF_OK) return rc == PMF_EBUSY ? PMF_ENOMEM : rc;
    // The work list keeps finished instances (their tiles exit at once), so
    // one captured superstep graph serves the whole solve.
    const int S = h->opt.steps_per_sync;
    const int64_t max_rounds = h->opt.max_supersteps / S + 4;
    int64_t done = 0;
    std::vector<int> fin;
    for (int64_t round = 0; done < (int64_t)subs.size(); ++round) {
        if (round > max_rounds) return PMF_ETIMEOUT;
        fin.clear();
        rc = run_steps(h, S, &fin, 1 << 16);
        if (rc != PMF_OK) return rc;
        done += (int64_t)fin.size();
        h->wl_dirty = false;
    }
    if (launch_finalize(d_sub_status, d_meta, n_inst, flows_out, status_out, h->stream) != 0) return PMF_EDEVICE;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return PMF_EDEVICE;
    return PMF_OK;
}

}  // namespace

namespace {

// One solved lambda of a breakpoint search: its flow, |S_min| and slope sum
// w(S_min) (the derivative of F on the piece where S_min is optimal).
struct BpPoint {
    int64_t F = 0, size = 0, w = 0;
};

// Every integer change point c in (lam_lo, lam_hi] of `base` (one instance,
// schedule unused), in increasing order, with every solved lambda in pts;
// exit_out (device, may be null) receives each pixel's first lambda outside
// S_min (lam_lo if never in it, lam_hi + 1 if it never leaves).  Leaves the
// arena tail in use: the caller releases it.
int integer_breakpoints(pmf_handle *h, const pmf_instance &base, int32_t lam_lo, int32_t lam_hi,
                        std::map<int32_t, BpPoint> &pts, std::vector<int32_t> &changes, int32_t *exit_out) {
    const int n = base.W * base.H;
    // the exit map is a running minimum over the solved lambdas: the smallest
    // solved lambda whose set lacks the pixel (every change point is solved,
    // and the set is constant between change points, so it is exact)
    if (exit_out && launch_fill_i32(exit_out, n, lam_hi + 1, h->stream) != 0) return PMF_EDEVICE;
    // Probes per round: the batched call solves them side by side, so a round
    // costs about as much as its slowest chunk until the device fills, and
    // fewer, wider rounds win.  The budget shrinks for large images so that
    // the round's state stays within 1 GiB.
    int budget = 64;
    for (pmf_instance I = base; budget > 2; budget /= 2) {
        I.L = budget;
        int64_t subs = 0;
        if (batch_pool_bytes(&I, 1, 1, h->tw, h->th, h->opt.gap != 0, &subs) <= ((size_t)1 << 30)) break;
    }
    // Solve the (ascending, distinct) lambdas of `lams` as the schedule of one
    // instance: the batched call splits it into warm-started chunks solved in
    // parallel.  The round's own device data (lambdas, flows, status, mask
    // statistics) sit at the end of the handle's arena, which is first grown to
    // hold them next to the largest layout the call can pick (every lambda a
    // chunk of its own), so that the call never moves it.  The masks are read
    // where the solve left them.
    auto solve = [&](const std::vector<int32_t> &lams) -> int {
        const int m = (int)lams.size();
        const size_t o_f = align_up(4 * (size_t)m), o_s = o_f + align_up(8 * (size_t)m), o_st = o_s + align_up(4),
                     T = o_st + align_up(16 * (size_t)m);
        pmf_instance I = base;
        I.L = m;
        int64_t subs = 0;
        const size_t pool1 = batch_pool_bytes(&I, 1, 1, h->tw, h->th, h->opt.gap != 0, &subs);
        const size_t need = control_bytes((int)subs, worklist_cap((int)subs, pool1)) + pool1;
        h->reserve_tail = 0;
        int rc = ensure_arena(h, need + T);
        if (rc != PMF_OK) return rc;
        h->reserve_tail = T;
        char *tail = h->arena + h->arena_bytes - T;
        int32_t *dl = (int32_t *)tail;
        int64_t *df = (int64_t *)(tail + o_f);
        int32_t *ds = (int32_t *)(tail + o_s);
        int64_t *dst = (int64_t *)(tail + o_st);
        if (hipMemcpyAsync(dl, lams.data(), 4 * (size_t)m, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
            hipMemsetAsync(dst, 0, 16 * (size_t)m, h->stream) != hipSuccess)
            return PMF_EDEVICE;
        I.lambdas = dl;
        rc = pmf_solve_batch(h, &I, 1, df, ds);
        if (rc != PMF_OK) return rc;
        int32_t st = PMF_OK;
        if (hipMemcpy(&st, ds, 4, hipMemcpyDeviceToHost) != hipSuccess) return PMF_EDEVICE;
        if (st != PMF_OK) return st;
        for (int i = 0; i < m; ++i) {
            int slot, k;
            rc = locate(h, 0, i, &slot, &k);
            if (rc != PMF_OK) return rc;
            const uint8_t *mask = (const uint8_t *)(h->base + h->slots[slot].masks + (size_t)k * n);
            if (launch_mask_stats(mask, n, base.snk_slope, base.seed, dst + 2 * i, h->stream) != 0) return PMF_EDEVICE;
            if (exit_out && launch_exit_min(mask, n, lams[i], exit_out, h->stream) != 0) return PMF_EDEVICE;
        }
        std::vector<int64_t> f(m), sw(2 * (size_t)m);
        if (hipMemcpyAsync(f.data(), df, 8 * (size_t)m, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
            hipMemcpyAsync(sw.data(), dst, 16 * (size_t)m, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            return PMF_EDEVICE;
        for (int i = 0; i < m; ++i) {
            BpPoint &q = pts[lams[i]];
            q.F = f[i];
            q.size = sw[2 * i];
            q.w = sw[2 * i + 1];
        }
        return PMF_OK;
    };
    // Up to k probes strictly inside (a, b), an interval whose end sets differ
    // (nested sets are equal exactly when their sizes are), into `out`.  When k
    // covers every integer inside, all of them.  Otherwise first the two
    // integers around the meeting point x of the end pieces of F,
    // F(a) + w_a (l - a) and F(b) + w_b (l - b): a single change point c in
    // (a, b] satisfies c - 1 < x <= c, so ceil(x) - 1 and ceil(x) isolate it
    // (the midpoint instead when w_a = w_b, which free pixels of slope 0
    // allow).  The rest are spread over (a, b), geometrically when a > 0, for
    // intervals that hold several change points.
    auto probes = [&](int32_t a, int32_t b, int k, std::vector<int32_t> &out) {
        if ((int64_t)b - a - 1 <= k) {
            for (int32_t x = a + 1; x < b; ++x) out.push_back(x);
            return;
        }
        std::vector<int32_t> mine;
        auto add = [&](int64_t x) {
            x = std::min<int64_t>(std::max<int64_t>(x, (int64_t)a + 1), (int64_t)b - 1);
            if (std::find(mine.begin(), mine.end(), (int32_t)x) == mine.end()) mine.push_back((int32_t)x);
        };
        const BpPoint &pa = pts[a], &pb = pts[b];
        if (pa.w > pb.w) {
            const long double x = ((long double)pb.F - pa.F + (long double)pa.w * a - (long double)pb.w * b) /
                                  (long double)(pa.w - pb.w);
            const int64_t c = (int64_t)std::ceil(x);
            add(c);
            add(c - 1);
        } else {
            add((int64_t)a + (b - a) / 2);
        }
        const int rest = k - (int)mine.size();
        for (int j = 1; j <= rest; ++j) {
            const double t = (double)j / (rest + 1);
            add(a > 0 ? (int64_t)std::llround(a * std::pow((double)b / a, t)) : (int64_t)a + (int64_t)((b - a) * t));
        }
        out.insert(out.end(), mine.begin(), mine.end());
    };
    std::vector<int32_t> ends = {lam_lo};
    if (lam_hi > lam_lo) ends.push_back(lam_hi);
    int rc = solve(ends);
    if (rc != PMF_OK) return rc;
    // Open intervals: consecutive solved lambdas whose sets differ.  One of
    // length 1 is a change point; the others share the round's probe budget.
    std::vector<std::pair<int32_t, int32_t>> open;
    if (lam_hi > lam_lo && pts[lam_lo].size != pts[lam_hi].size) open.push_back({lam_lo, lam_hi});
    changes.clear();
    while (!open.empty()) {
        std::vector<std::pair<int32_t, int32_t>> live;
        for (const auto &iv : open) {
            if (iv.second - iv.first == 1)
                changes.push_back(iv.second);
            else
                live.push_back(iv);
        }
        open.clear();
        if (live.empty()) break;
        const int k = std::max(2, budget / (int)live.size());
        std::vector<int32_t> mids;
        for (const auto &iv : live) probes(iv.first, iv.second, k, mids);
        std::sort(mids.begin(), mids.end());
        mids.erase(std::unique(mids.begin(), mids.end()), mids.end());
        rc = solve(mids);
        if (rc != PMF_OK) return rc;
        for (const auto &iv : live) {
            // the solved lambdas inside (a, b) cut it into pieces
            auto it = pts.upper_bound(iv.first);
            int32_t prev = iv.first;
            for (; it != pts.end() && it->first <= iv.second; ++it) {
                if (pts[prev].size != it->second.size) open.push_back({prev, it->first});
                prev = it->first;
            }
        }
    }
    std::sort(changes.begin(), changes.end());
    changes.erase(std::unique(changes.begin(), changes.end()), changes.end());
    return PMF_OK;
}

// The instance of a breakpoint search: one lambda, its schedule supplied by
// the search (only the pointer's presence is checked here).
int breakpoint_base(const pmf_instance *inst, int32_t lam_lo, int32_t lam_hi, pmf_instance *base) {
    if (!inst || lam_lo < 0 || lam_hi < lam_lo) return PMF_EINVAL;
    if (lam_hi == INT32_MAX) return PMF_EINVAL;  // lam_hi + 1 marks pixels that never leave
    *base = *inst;
    base->L = 1;
    base->lambdas = nullptr;
    pmf_instance chk = *base;
    chk.lambdas = &lam_lo;
    return check_instance(chk) != PMF_OK ? PMF_EINVAL : PMF_OK;
}

}  // namespace

extern "C" {

int pmf_solve_batch(pmf_handle *h, const pmf_instance *inst, int32_t n_inst, int64_t *flows_out,
                    int32_t *status_out) {
    if (!h) return PMF_EINVAL;
    (void)finish_async(h);
    return solve_batch(h, inst, n_inst, flows_out, status_out);
}

int pmf_solve_batch_async(pmf_handle *h, const pmf_instance *inst, int32_t n_inst, int64_t *flows_out,
                          int32_t *status_out) {
    if (!h) return PMF_EINVAL;
    (void)finish_async(h);
    if (n_inst < 0 || (n_inst > 0 && (!inst || !flows_out))) return PMF_EINVAL;
    const int rc = pmf_check_instances(inst, n_inst, nullptr);
    if (rc != PMF_OK) return rc;
    h->async_inst.assign(inst, inst + n_inst);
    h->async_done.store(0);
    try {
        h->worker = std::thread([h, n_inst, flows_out, status_out]() {
            int r = hipSetDevice(h->device) == hipSuccess ? PMF_OK : PMF_EDEVICE;
            if (r == PMF_OK) r = solve_batch(h, h->async_inst.data(), n_inst, flows_out, status_out);
            h->async_rc = r;
            h->async_done.store(1);
        });
    } catch (...) {
        h->async_done.store(1);
        return PMF_EDEVICE;
    }
    return PMF_OK;
}

int pmf_wait(pmf_handle *h) {
    if (!h) return PMF_EINVAL;
    return finish_async(h);
}

int pmf_query_done(pmf_handle *h, int32_t *done) {
    if (!h || !done) return PMF_EINVAL;
    *done = h->async_done.load();
    return PMF_OK;
}

int pmf_solve_batch_noalloc(pmf_handle *h, const pmf_instance *inst, int32_t n_inst, int64_t *flows_out,
                            int32_t *status_out) {
    if (!h) return PMF_EINVAL;
    (void)finish_async(h);
    // timing mode keeps events and counters of its own: not available here
    if (h->opt.timing != 0) return PMF_EINVAL;
    if (!h->scratch_dev) return PMF_EDEVICE;
    const int rc = solve_batch(h, inst, n_inst, flows_out, status_out, h->scratch_dev, PMF_NOALLOC_BYTES);
    return rc == PMF_ENOMEM ? PMF_ELIMIT : rc;
}

int pmf_extract_cut(pmf_handle *h, int32_t inst, int32_t lambda_idx, uint8_t *mask_out) {
    if (!h || !mask_out) return PMF_EINVAL;
    (void)finish_async(h);
    if (!h->open) return PMF_ENOTSOLVED;
    int slot, k;
    const int rc = locate(h, inst, lambda_idx, &slot, &k);
    if (rc != PMF_OK) return rc;
    const Slot &s = h->slots[slot];
    if (!s.live || !s.finished || s.done_k <= k) return PMF_ENOTSOLVED;
    const size_t px = (size_t)s.W * s.H;
    const char *src = h->base + s.masks + (size_t)k * px;
    if (hipMemcpyAsync(mask_out, src, px, hipMemcpyDeviceToDevice, h->stream) != hipSuccess) return PMF_EDEVICE;
    return PMF_OK;
}

int pmf_extract_levels(pmf_handle *h, int32_t inst, uint8_t *levels_out) {
    if (!h || !levels_out) return PMF_EINVAL;
    (void)finish_async(h);
    if (!h->open) return PMF_ENOTSOLVED;
    int first, last;
    if (h->batch) {
        if (inst < 0 || inst >= (int)h->user_L.size()) return PMF_ERANGE;
        if (h->user_L[inst] > 255) return PMF_ERANGE;
        first = h->user_first[inst];
        last = h->user_first[inst + 1];
    } else {
        if (inst < 0 || inst >= h->max_slots || !h->slots[inst].live) return PMF_ERANGE;
        if (h->slots[inst].L > 255) return PMF_ERANGE;
        first = inst;
        last = inst + 1;
    }
    for (int sl = first; sl < last; ++sl) {
        const Slot &s = h->slots[sl];
        if (!s.live || !s.finished || s.done_k < s.L) return PMF_ENOTSOLVED;
    }
    // every chunk adds the lambdas it holds (the sets are nested across chunks too)
    for (int sl = first; sl < last; ++sl) {
        const Slot &s = h->slots[sl];
        const uint8_t *masks = (const uint8_t *)(h->base + s.masks);
        if (launch_levels(masks, s.L, s.W * s.H, levels_out, sl > first, h->stream) != 0) return PMF_EDEVICE;
    }
    return PMF_OK;
}

int pmf_session_open(pmf_handle *h, int32_t max_slots, size_t pool_bytes) {
    if (!h || max_slots < 1) return PMF_EINVAL;
    (void)finish_async(h);
    h->batch = false;
    if (pool_bytes == 0) {
        size_t avail = 0;
        if (!h->own_arena) {
            avail = h->arena_bytes;
        } else if (h->opt.mem_budget > 0) {
            avail = (size_t)h->opt.mem_budget;
        } else {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) return PMF_EDEVICE;
            avail = fr / 2 + h->arena_bytes;
        }
        // the control area grows with the pool (work list); leave room for it
        const size_t ctl0 = control_bytes(max_slots, (size_t)max_slots);
        if (avail <= ctl0 + (1 << 20)) return PMF_ENOMEM;
        pool_bytes = (avail - ctl0) / 129 * 128;
        while (pool_bytes > 0 && control_bytes(max_slots, worklist_cap(max_slots, pool_bytes)) + pool_bytes > avail)
            pool_bytes -= std::min(pool_bytes, (size_t)1 << 20);
    }
    return open_session(h, max_slots, pool_bytes);
}

int pmf_session_submit(pmf_handle *h, const pmf_instance *inst, int32_t n_inst, int64_t *flows_out,
                       int32_t *status_out, int32_t *ids_out) {
    if (!h) return PMF_EINVAL;
    (void)finish_async(h);
    return submit(h, inst, n_inst, flows_out, status_out, ids_out);
}

int pmf_session_step(pmf_handle *h, int32_t supersteps, int32_t *done_ids, int32_t max_ids, int32_t *n_done) {
    if (!h || supersteps < 1 || supersteps > (1 << 16) || max_ids < 0 || (max_ids > 0 && !done_ids))
        return PMF_EINVAL;
    if (n_done) *n_done = 0;
    (void)finish_async(h);
    if (!h->open) return PMF_EINVAL;
    std::vector<int> fin;
    const int rc = run_steps(h, supersteps, &fin);
    if (rc != PMF_OK) return rc;
    const int n = std::min((int)fin.size(), (int)max_ids);
    for (int i = 0; i < n; ++i) done_ids[i] = fin[i];
    if (n_done) *n_done = (int32_t)fin.size();
    return PMF_OK;
}

int pmf_session_release(pmf_handle *h, int32_t id) {
    if (!h) return PMF_EINVAL;
    (void)finish_async(h);
    if (!h->open) return PMF_EINVAL;
    if (id < 0 || id >= h->max_slots || !h->slots[id].live) return PMF_ERANGE;
    Slot &s = h->slots[id];
    if (!s.finished) {
        // cancel: the slot goes idle before its memory can be reused
        InstState idle;
        std::memset(&idle, 0, sizeof(idle));
        if (hipMemcpyAsync(h->P.st + id, &idle, sizeof(idle), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            return PMF_EDEVICE;
        h->wl_dirty = true;
    }
    h->pool.release(s.off, s.bytes);
    s = Slot();
    h->free_slots.push_back(id);
    std::sort(h->free_slots.begin(), h->free_slots.end(), std::greater<int>());
    return PMF_OK;
}

int pmf_session_query(pmf_handle *h, pmf_session_info *out) {
    if (!h || !out) return PMF_EINVAL;
    (void)finish_async(h);
    std::memset(out, 0, sizeof(*out));
    if (!h->open) return PMF_OK;
    out->free_bytes = (int64_t)h->pool.free_bytes();
    out->largest_free = (int64_t)h->pool.largest();
    out->free_slots = (int32_t)h->free_slots.size();
    for (const Slot &s : h->slots) {
        out->admitted += s.live;
        out->running += s.live && !s.finished;
    }
    return PMF_OK;
}

int pmf_slot_stats(pmf_handle *h, int64_t *out, int32_t max_slots, int32_t *n_slots) {
    if (!h || max_slots < 0 || (max_slots > 0 && !out)) return PMF_EINVAL;
    (void)finish_async(h);
    const int n = h->open ? h->max_slots : 0;
    if (n_slots) *n_slots = n;
    for (int i = 0; i < std::min(n, (int)max_slots); ++i) {
        int64_t *o = out + 8 * (size_t)i;
        const Slot &s = h->slots[i];
        std::memset(o, 0, 8 * sizeof(int64_t));
        if (!s.live || !s.finished) continue;
        const InstState &x = h->ext ? h->host_state[i] : h->pinned_state[i];
        o[0] = 1;
        o[1] = x.steps;
        o[2] = x.sweeps;
        o[3] = x.relabels;
        o[4] = x.passes;
        o[5] = x.k;
        o[6] = x.px_sweep;
        o[7] = x.px_relabel;
    }
    return PMF_OK;
}

int pmf_get_stats(pmf_handle *h, pmf_stats *out) {
    if (!h || !out) return PMF_EINVAL;
    (void)finish_async(h);
    *out = h->stats;
    return PMF_OK;
}

int64_t pmf_get_trace(pmf_handle *h, int64_t *out, int64_t max_rows) {
    if (!h || max_rows < 0 || (max_rows > 0 && !out)) return -(int64_t)PMF_EINVAL;
    (void)finish_async(h);
    const int64_t rows = (int64_t)h->trace.size() / PMF_TRACE_COLS;
    const int64_t n = std::min(rows, max_rows);
    if (n > 0) std::copy(h->trace.begin(), h->trace.begin() + n * PMF_TRACE_COLS, out);
    return rows;
}

int pmf_parametric(pmf_handle *h, const pmf_instance *inst, int32_t lam_lo, int32_t lam_hi, int32_t *bp_out,
                   int64_t *f_out, int32_t max_bp, int32_t *n_bp, int32_t *exit_out) {
    if (!h || !inst || !n_bp || max_bp < 0 || (max_bp > 0 && !bp_out)) return PMF_EINVAL;
    pmf_instance base;
    if (breakpoint_base(inst, lam_lo, lam_hi, &base) != PMF_OK) return PMF_EINVAL;
    (void)finish_async(h);
    (void)hipStreamSynchronize(h->stream);
    h->open = false;  // the search's own buffers overwrite the last solve's memory
    *n_bp = 0;
    std::map<int32_t, BpPoint> pts;
    std::vector<int32_t> changes;
    const int rc = integer_breakpoints(h, base, lam_lo, lam_hi, pts, changes, exit_out);
    (void)hipStreamSynchronize(h->stream);
    h->reserve_tail = 0;
    if (rc != PMF_OK) return rc;
    *n_bp = (int32_t)changes.size();
    for (int i = 0; i < (int)changes.size() && i < max_bp; ++i) bp_out[i] = changes[i];
    if (f_out) {
        f_out[0] = pts[lam_lo].F;
        for (int i = 0; i < (int)changes.size() && i < max_bp; ++i) f_out[i + 1] = pts[changes[i]].F;
    }
    return (int)changes.size() > max_bp ? PMF_ERANGE : PMF_OK;
}

int pmf_breakpoints(pmf_handle *h, const pmf_instance *inst, int32_t lam_lo, int32_t lam_hi, int64_t *bp_num,
                    int64_t *bp_den, int64_t *piece_a, int64_t *piece_w, int32_t max_bp, int32_t *n_bp,
                    int32_t *exit_out) {
    if (!h || !inst || !n_bp || !exit_out || !piece_a || !piece_w || max_bp < 0 ||
        (max_bp > 0 && (!bp_num || !bp_den)))
        return PMF_EINVAL;
    pmf_instance base;
    if (breakpoint_base(inst, lam_lo, lam_hi, &base) != PMF_OK) return PMF_EINVAL;
    (void)finish_async(h);
    (void)hipStreamSynchronize(h->stream);
    h->open = false;  // the search's own buffers overwrite the last solve's memory
    *n_bp = 0;
    auto release = [&](int code) {
        (void)hipStreamSynchronize(h->stream);
        h->reserve_tail = 0;
        return code;
    };
    // 1. every integer change point c (S_min(c - 1) != S_min(c)), with the
    // integer exit map in exit_out: S_min(l) = {p : exit[p] > l} for every
    // integer l of the range
    std::map<int32_t, BpPoint> pts;
    std::vector<int32_t> changes;
    int rc = integer_breakpoints(h, base, lam_lo, lam_hi, pts, changes, exit_out);
    if (rc != PMF_OK) return release(rc);
    (void)hipStreamSynchronize(h->stream);
    h->reserve_tail = 0;
    struct Line {  // cut cost a + w * lambda of one source set
        int64_t a, w;
    };
    auto line_at = [&](int32_t lam, Line *out) {
        const auto it = pts.find(lam);
        if (it == pts.end()) return false;
        *out = Line{it->second.F - it->second.w * (int64_t)lam, it->second.w};
        return true;
    };
    const int W = base.W, H = base.H, K = base.K, n = W * H, k = (int)changes.size();
    Line first;
    if (!line_at(lam_lo, &first)) return release(PMF_EDEVICE);
    piece_a[0] = first.a;
    piece_w[0] = first.w;
    if (k == 0) {
        if (launch_exit_pieces_init(exit_out, n, lam_lo, lam_hi, 1, h->stream) != 0) return release(PMF_EDEVICE);
        return release(PMF_OK);
    }
    // 2. the box of D_c = S_min(c - 1) \ S_min(c) = {p : exit[p] == c}
    std::vector<int32_t> box(4 * (size_t)k);
    {
        const size_t o_box = align_up(4 * (size_t)k), T = o_box + align_up(16 * (size_t)k);
        rc = ensure_arena(h, T);
        if (rc != PMF_OK) return release(rc);
        char *tail = h->arena + h->arena_bytes - T;
        if (hipMemcpyAsync(tail, changes.data(), 4 * (size_t)k, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
            launch_change_boxes(exit_out, W, H, (const int32_t *)tail, k, (int32_t *)(tail + o_box), h->stream) != 0 ||
            hipMemcpyAsync(box.data(), tail + o_box, 16 * (size_t)k, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            return release(PMF_EDEVICE);
    }
    struct Interval {
        int32_t c;
        int x0, y0, w, h;
        int64_t a;
        size_t o_planes, o_ep, o_eq, o_stats;
        int64_t st[kCsCount];
        Line fix;  // full-problem line = contracted line + fix
    };
    std::vector<Interval> iv(k);
    size_t P = 0;
    int64_t amax = 0;
    int wmax = 0, hmax = 0;
    for (int i = 0; i < k; ++i) {
        Interval &I = iv[i];
        I.c = changes[i];
        I.x0 = box[4 * i];
        I.y0 = box[4 * i + 1];
        if (box[4 * i + 2] < I.x0 || box[4 * i + 3] < I.y0) return release(PMF_EDEVICE);  // D is never empty
        I.w = box[4 * i + 2] - I.x0 + 1;
        I.h = box[4 * i + 3] - I.y0 + 1;
        I.a = (int64_t)I.w * I.h;
        I.o_planes = P;
        P = align_up(P + 4 * (size_t)(K + 3) * I.a);
        I.o_ep = P;
        P = align_up(P + 4 * (size_t)I.a);
        I.o_eq = P;
        P = align_up(P + 4 * (size_t)I.a);
        I.o_stats = P;
        P = align_up(P + 8 * (size_t)kCsCount);
        amax = std::max(amax, I.a);
        wmax = std::max(wmax, I.w);
        hmax = std::max(hmax, I.h);
    }
    // 3. device memory: the contracted problems (kept to the end), then per
    // round up to R scaled copies with their lambdas, flows, statuses and set
    // statistics, and the pool of a batch of R probes of the largest box
    const size_t probe_planes = align_up(4 * (size_t)(K + 2) * amax);
    auto round_pool = [&](int m) {
        pmf_instance M = base;
        M.W = wmax;
        M.H = hmax;
        std::vector<pmf_instance> v((size_t)m, M);
        int64_t subs = 0;
        const size_t pool = batch_pool_bytes(v.data(), m, 1, h->tw, h->th, h->opt.gap != 0, &subs);
        return control_bytes((int)subs, worklist_cap((int)subs, pool)) + pool;
    };
    auto round_scratch = [&](int m) {
        return (size_t)m * probe_planes + align_up(4 * (size_t)m) + align_up(8 * (size_t)m) +
               align_up(4 * (size_t)m) + align_up(16 * (size_t)m);
    };
    int R = 64;
    while (R > 1 && round_pool(R) + round_scratch(R) > ((size_t)1 << 30)) R /= 2;
    const size_t T = P + round_scratch(R);
    rc = ensure_arena(h, round_pool(R) + T);
    if (rc != PMF_OK) return release(rc);
    h->reserve_tail = T;
    char *pers = h->arena + h->arena_bytes - T, *scr = pers + P;
    const size_t o_l = (size_t)R * probe_planes, o_f = o_l + align_up(4 * (size_t)R),
                 o_s = o_f + align_up(8 * (size_t)R), o_st = o_s + align_up(4 * (size_t)R);
    int32_t *dl = (int32_t *)(scr + o_l), *ds = (int32_t *)(scr + o_s);
    int64_t *df = (int64_t *)(scr + o_f), *dst = (int64_t *)(scr + o_st);
    // 4. contract each interval's problem to its changing pixels
    for (int i = 0; i < k; ++i) {
        Interval &I = iv[i];
        if (launch_contract(base.nlink, base.cap_src, base.cap_snk0, base.snk_slope, base.seed, W, H, K, exit_out,
                            I.c, I.x0, I.y0, I.w, I.h, (int32_t *)(pers + I.o_planes), (int32_t *)(pers + I.o_ep),
                            (int32_t *)(pers + I.o_eq), (int64_t *)(pers + I.o_stats), h->stream) != 0 ||
            hipMemcpyAsync(I.st, pers + I.o_stats, 8 * (size_t)kCsCount, hipMemcpyDeviceToHost, h->stream) !=
                hipSuccess)
            return release(PMF_EDEVICE);
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) return release(PMF_EDEVICE);
    // the two end lines of an interval in the contracted problem: all of D
    // in the source set (cost sum c0 + lambda * sum slope) and none of it
    // (cost sum cs); the pixels fixed by the contraction add the same line
    // to every set, read off the full problem's lines at c - 1 and c
    struct Pair {
        int iv;
        Line L, R;       // L optimal left of the meeting point, R right of it
        int64_t rp, rq;  // R is optimal at rp / rq
    };
    struct Found {
        int iv;
        int64_t p, q;
        Line L, R;
    };
    std::vector<Pair> pend;
    std::vector<Found> found;
    for (int i = 0; i < k; ++i) {
        Interval &I = iv[i];
        if (I.st[kCsSeeds] != 0) return release(PMF_ERANGE);  // capacities at INF: no finite contraction
        const Line Lc{I.st[kCsSumC0], I.st[kCsSumSl]}, Rc{I.st[kCsSumCs], 0};
        Line Lf, Rf;
        if (!line_at(I.c - 1, &Lf) || !line_at(I.c, &Rf)) return release(PMF_EDEVICE);
        I.fix = Line{Lf.a - Lc.a, Lf.w - Lc.w};
        if (Rf.a != Rc.a + I.fix.a || Rf.w != Rc.w + I.fix.w) return release(PMF_EDEVICE);
        pend.push_back(Pair{i, Lc, Rc, I.c, 1});
    }
    // 5. rounds: each pending pair (L, R) meets at x = p / q; if F(x) is on
    // both lines, x is the only breakpoint between them, else the minimal
    // set at x gives a new line M and the pairs (L, M) and (M, R).  F(x) and
    // S_min(x) come from the contracted problem with every capacity
    // multiplied by q, solved at the integer lambda p.
    struct Probe {
        Pair pr;
        int32_t p, q;
    };
    int64_t probes_total = 0;
    while (!pend.empty()) {
        std::vector<Probe> todo;
        for (const Pair &pr : pend) {
            const int64_t num = pr.R.a - pr.L.a, den = pr.L.w - pr.R.w;
            if (den <= 0 || num <= 0) return release(PMF_EDEVICE);
            const int64_t g = std::gcd(num, den), p = num / g, q = den / g;
            const Interval &I = iv[pr.iv];
            if ((__int128)p <= (__int128)(I.c - 1) * q || (__int128)p > (__int128)I.c * q)
                return release(PMF_EDEVICE);
            if ((__int128)p * pr.rq > (__int128)pr.rp * q) return release(PMF_EDEVICE);  // past R's point
            if ((__int128)p * pr.rq == (__int128)pr.rp * q) {  // at R's own point: F(x) is known
                found.push_back(Found{pr.iv, p, q, pr.L, pr.R});
                continue;
            }
            const __int128 lim = PMF_INF;
            if (p > INT32_MAX || q > lim || (__int128)q * I.st[kCsMaxCs] > lim ||
                (__int128)q * I.st[kCsMaxNl] > PMF_NLINK_MAX(K) ||
                (__int128)q * I.st[kCsMaxC0] + (__int128)I.st[kCsMaxSl] * p > lim)
                return release(PMF_ERANGE);
            todo.push_back(Probe{pr, (int32_t)p, (int32_t)q});
        }
        probes_total += (int64_t)todo.size();
        if (probes_total > ((int64_t)1 << 22)) return release(PMF_ETIMEOUT);
        std::vector<Pair> next;
        for (size_t b0 = 0; b0 < todo.size(); b0 += (size_t)R) {
            const int m = (int)std::min<size_t>((size_t)R, todo.size() - b0);
            std::vector<pmf_instance> pi((size_t)m);
            std::vector<int32_t> lam((size_t)m), sts((size_t)m);
            for (int j = 0; j < m; ++j) {
                const Probe &pb = todo[b0 + j];
                const Interval &I = iv[pb.pr.iv];
                const int32_t *src = (const int32_t *)(pers + I.o_planes);
                int32_t *dstp = (int32_t *)(scr + (size_t)j * probe_planes);
                if (launch_scale(src, (int64_t)(K + 2) * I.a, pb.q, dstp, h->stream) != 0)
                    return release(PMF_EDEVICE);
                pmf_instance &Q = pi[j];
                Q = base;
                Q.W = I.w;
                Q.H = I.h;
                Q.L = 1;
                Q.nlink = dstp;
                Q.cap_src = dstp + (size_t)K * I.a;
                Q.cap_snk0 = dstp + (size_t)(K + 1) * I.a;
                Q.snk_slope = src + (size_t)(K + 2) * I.a;
                Q.seed = nullptr;
                Q.lambdas = dl + j;
                lam[j] = pb.p;
            }
            {
                // the batch must fit in front of the tail: a larger arena
                // would be a new allocation, and the tail would move
                int64_t subs = 0;
                const size_t pool = batch_pool_bytes(pi.data(), m, 1, h->tw, h->th, h->opt.gap != 0, &subs);
                if (control_bytes((int)subs, worklist_cap((int)subs, pool)) + pool + T > h->arena_bytes)
                    return release(PMF_ENOMEM);
            }
            if (hipMemcpyAsync(dl, lam.data(), 4 * (size_t)m, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
                hipMemsetAsync(dst, 0, 16 * (size_t)m, h->stream) != hipSuccess)
                return release(PMF_EDEVICE);
            // the contracted probes hold no seeds and are solved as given (the
            // orientation rule is tuned for seeded images)
            const int32_t orient = h->opt.orientation;
            h->opt.orientation = kOrientAsGiven;
            rc = pmf_solve_batch(h, pi.data(), m, df, ds);
            h->opt.orientation = orient;
            if (rc != PMF_OK) return release(rc);
            if (hipMemcpy(sts.data(), ds, 4 * (size_t)m, hipMemcpyDeviceToHost) != hipSuccess)
                return release(PMF_EDEVICE);
            for (int j = 0; j < m; ++j)
                if (sts[j] != PMF_OK) return release(sts[j]);
            for (int j = 0; j < m; ++j) {
                const Probe &pb = todo[b0 + j];
                const Interval &I = iv[pb.pr.iv];
                int slot, kk;
                rc = locate(h, j, 0, &slot, &kk);
                if (rc != PMF_OK) return release(rc);
                const uint8_t *mask = (const uint8_t *)(h->base + h->slots[slot].masks + (size_t)kk * I.a);
                if (launch_mask_stats(mask, (int)I.a, pi[j].snk_slope, nullptr, dst + 2 * j, h->stream) != 0 ||
                    launch_exit_rational(mask, (int)I.a, pb.p, pb.q, (int32_t *)(pers + I.o_ep),
                                         (int32_t *)(pers + I.o_eq), h->stream) != 0)
                    return release(PMF_EDEVICE);
            }
            std::vector<int64_t> f((size_t)m), sw(2 * (size_t)m);
            if (hipMemcpyAsync(f.data(), df, 8 * (size_t)m, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
                hipMemcpyAsync(sw.data(), dst, 16 * (size_t)m, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
                hipStreamSynchronize(h->stream) != hipSuccess)
                return release(PMF_EDEVICE);
            for (int j = 0; j < m; ++j) {
                const Probe &pb = todo[b0 + j];
                const Pair &pr = pb.pr;
                const __int128 on_l = (__int128)pb.q * pr.L.a + (__int128)pr.L.w * pb.p;
                if (f[j] == on_l) {
                    found.push_back(Found{pr.iv, pb.p, pb.q, pr.L, pr.R});
                } else if (f[j] < on_l) {
                    const int64_t wm = sw[2 * j + 1];
                    const __int128 am = (__int128)f[j] - (__int128)wm * pb.p;
                    if (am % pb.q != 0) return release(PMF_EDEVICE);
                    const Line M{(int64_t)(am / pb.q), wm};
                    next.push_back(Pair{pr.iv, pr.L, M, pb.p, pb.q});
                    next.push_back(Pair{pr.iv, M, pr.R, pr.rp, pr.rq});
                } else {
                    return release(PMF_EDEVICE);  // a cut cheaper than the minimum
                }
            }
        }
        pend.swap(next);
    }
    // 6. the breakpoints in increasing order, each piece's line in the full
    // problem, and every pixel's exit piece
    std::sort(found.begin(), found.end(), [](const Found &x, const Found &y) {
        if (x.iv != y.iv) return x.iv < y.iv;
        return (__int128)x.p * y.q < (__int128)y.p * x.q;
    });
    const int nb = (int)found.size();
    Line cur = first;
    std::vector<int64_t> table(2 * (size_t)nb);
    std::vector<int> start(k + 1, 0);
    for (int j = 0; j < nb; ++j) {
        const Found &fd = found[j];
        const Line &fx = iv[fd.iv].fix;
        const Line Lf{fd.L.a + fx.a, fd.L.w + fx.w}, Rf{fd.R.a + fx.a, fd.R.w + fx.w};
        if (Lf.a != cur.a || Lf.w != cur.w) return release(PMF_EDEVICE);
        if (j < max_bp) {
            bp_num[j] = fd.p;
            bp_den[j] = fd.q;
            piece_a[j + 1] = Rf.a;
            piece_w[j + 1] = Rf.w;
        }
        table[2 * j] = fd.p;
        table[2 * j + 1] = fd.q;
        start[fd.iv + 1] = j + 1;
        cur = Rf;
    }
    for (int i = 0; i < k; ++i) start[i + 1] = std::max(start[i + 1], start[i]);
    *n_bp = nb;
    if (launch_exit_pieces_init(exit_out, n, lam_lo, lam_hi, nb + 1, h->stream) != 0) return release(PMF_EDEVICE);
    // each interval's breakpoints go to the start of the round area before
    // its placement kernel (stream order keeps the previous one's reads)
    const size_t room = (size_t)R * probe_planes;
    size_t at = 0;
    for (int i = 0; i < k; ++i) {
        const Interval &I = iv[i];
        const int cnt = start[i + 1] - start[i];
        const size_t bytes = 16 * (size_t)cnt;
        if (at + bytes > room) at = 0;
        if (bytes > room) return release(PMF_ENOMEM);
        int64_t *dtab = (int64_t *)(scr + at);
        if (hipMemcpyAsync(dtab, table.data() + 2 * (size_t)start[i], bytes, hipMemcpyHostToDevice, h->stream) !=
                hipSuccess ||
            launch_exit_place((const int32_t *)(pers + I.o_ep), (const int32_t *)(pers + I.o_eq), I.x0, I.y0, I.w,
                              I.h, W, dtab, cnt, start[i], exit_out, h->stream) != 0)
            return release(PMF_EDEVICE);
        at = align_up(at + bytes);
    }
    return release(nb > max_bp ? PMF_ERANGE : PMF_OK);
}

int pmf_destroy(pmf_handle *h) {
    if (!h) return PMF_EINVAL;
    (void)finish_async(h);
    (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    if (h->own_arena && h->arena) (void)hipFree(h->arena);
    if (h->pinned) (void)hipHostFree(h->pinned);
    if (h->pinned_params) (void)hipHostFree(h->pinned_params);
    if (h->pinned_ring) (void)hipHostFree(h->pinned_ring);
    if (h->pinned_state) (void)hipHostFree(h->pinned_state);
    if (h->capture) (void)hipStreamDestroy(h->capture);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    for (hipEvent_t e : h->kev)
        if (e) (void)hipEventDestroy(e);
    if (h->trace_lists) (void)hipFree(h->trace_lists);
    if (h->kpx) (void)hipFree(h->kpx);
    delete h;
    return PMF_OK;
}

}  // extern "C"
