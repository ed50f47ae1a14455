// Host side of libpmf: argument validation, device memory layout, packing of
// instances into one tile space, and the superstep launch loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "pmf.h"
#include "pmf_internal.h"

using namespace pmf;

namespace {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
    size_t desc, st, tile_slot, tile_local, tile_act, tile_chg, tile_cnt, ctl;
    std::vector<size_t> r, e, rt, h, inbox, rmask, masks;
    size_t total = 0;
    int32_t ntiles = 0;
    std::vector<int32_t> tiles_x, tiles_y, tile0;
};

void tile_dims(const pmf_options &o, int *tw, int *th) {
    *tw = o.tile_w == 32 ? 32 : 64;
    *th = 1024 / *tw;
}

bool valid_options(const pmf_options &o) {
    if (o.tile_w != 0 && o.tile_w != 32 && o.tile_w != 64) return false;
    if (o.tile_h != 0 && o.tile_w != 0 && o.tile_w * o.tile_h != 1024) return false;
    if (o.inner_iters < 1 || o.inner_iters > 4096) return false;
    if (o.sweeps_per_relabel < 1 || o.sweeps_per_relabel > 1 << 20) return false;
    if (o.local_bfs_iters < 1 || o.local_bfs_iters > 1 << 20) return false;
    if (o.steps_per_sync < 1 || o.steps_per_sync > 1 << 16) return false;
    if (o.max_supersteps < 1) return false;
    if (o.order != 0 && o.order != 1) return false;
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

// Packing order: FIFO keeps the caller's order; LPT puts the instances with
// the most pixel-lambdas first so that the largest work is dispatched first
// (the "largest processing time first" rule, Sec. 3.3.1).
std::vector<int> packing_order(const pmf_instance *inst, int n, int order) {
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    if (order == 1) {
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            return (int64_t)inst[a].W * inst[a].H * inst[a].L > (int64_t)inst[b].W * inst[b].H * inst[b].L;
        });
    }
    return idx;
}

Layout plan(const pmf_instance *inst, int n, const pmf_options &o) {
    int tw, th;
    tile_dims(o, &tw, &th);
    Layout L;
    L.tiles_x.resize(n);
    L.tiles_y.resize(n);
    L.tile0.resize(n);
    std::vector<int> ord = packing_order(inst, n, o.order);
    int64_t t = 0;
    for (int i : ord) {
        L.tiles_x[i] = (inst[i].W + tw - 1) / tw;
        L.tiles_y[i] = (inst[i].H + th - 1) / th;
        L.tile0[i] = (int32_t)t;
        t += (int64_t)L.tiles_x[i] * L.tiles_y[i];
    }
    L.ntiles = (int32_t)t;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.desc = take(sizeof(InstDesc) * (size_t)n);
    L.st = take(sizeof(InstState) * (size_t)n);
    L.tile_slot = take(sizeof(int32_t) * (size_t)t);
    L.tile_local = take(sizeof(int32_t) * (size_t)t);
    L.tile_act = take(sizeof(uint32_t) * (size_t)t);
    L.tile_chg = take(2 * (size_t)t);
    L.tile_cnt = take(sizeof(int32_t) * (size_t)t);
    L.ctl = take(64);
    for (int i = 0; i < n; ++i) {
        const size_t px = (size_t)inst[i].W * inst[i].H, K = (size_t)inst[i].K;
        L.r.push_back(take(4 * K * px));
        L.e.push_back(take(4 * px));
        L.rt.push_back(take(4 * px));
        L.h.push_back(take(4 * px));
        L.inbox.push_back(take(4 * K * px));
        L.rmask.push_back(take(2 * px));
        L.masks.push_back(take((size_t)inst[i].L * px));
    }
    L.total = off;
    return L;
}

}  // namespace

struct pmf_handle {
    pmf_options opt;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    int device = 0;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    bool own_arena = true;
    int32_t *pinned = nullptr;  // host-visible completion counter
    // last solve
    bool solved = false;
    int n_inst = 0;
    std::vector<int32_t> W, H, L;
    std::vector<size_t> masks_off;
    std::vector<InstState> final_state;
    pmf_stats stats;
    hipGraphExec_t graph = nullptr;
};

namespace {

int ensure_arena(pmf_handle *h, size_t need) {
    if (need <= h->arena_bytes) return PMF_OK;
    if (!h->own_arena) return PMF_ENOMEM;
    if (h->opt.mem_budget > 0 && (int64_t)need > h->opt.mem_budget) return PMF_ENOMEM;
    if (h->arena) {
        (void)hipStreamSynchronize(h->stream);
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

void drop_graph(pmf_handle *h) {
    if (h->graph) {
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
}

}  // namespace

extern "C" {

void pmf_default_options(pmf_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tile_w = 64;
    o->tile_h = 16;
    o->inner_iters = 16;
    o->sweeps_per_relabel = 4;
    o->local_bfs_iters = 64;
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
        case PMF_EBUSY: return "no free slot";
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
    if (o.tile_w == 0) o.tile_w = 64;
    if (!valid_options(o)) return PMF_EINVAL;
    if (workspace && ws_bytes == 0) return PMF_EINVAL;
    pmf_handle *h = new (std::nothrow) pmf_handle();
    if (!h) return PMF_ENOMEM;
    h->opt = o;
    h->stream = (hipStream_t)stream;
    std::memset(&h->stats, 0, sizeof(h->stats));
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return PMF_EDEVICE;
    }
    if (workspace) {
        h->arena = (char *)workspace;
        h->arena_bytes = ws_bytes;
        h->own_arena = false;
    }
    if (hipHostMalloc((void **)&h->pinned, 64, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return PMF_EDEVICE;
    }
    if (hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking) != hipSuccess) {
        (void)hipHostFree(h->pinned);
        delete h;
        return PMF_EDEVICE;
    }
    *out = h;
    return PMF_OK;
}

int pmf_query_bytes(const pmf_instance *inst, int32_t n, const pmf_options *opt, size_t *bytes) {
    if (!bytes || n < 0 || (n > 0 && !inst)) return PMF_EINVAL;
    pmf_options o;
    if (opt)
        o = *opt;
    else
        pmf_default_options(&o);
    for (int i = 0; i < n; ++i)
        if (check_instance(inst[i]) != PMF_OK) return PMF_EINVAL;
    *bytes = plan(inst, n, o).total;
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

int pmf_solve_batch(pmf_handle *h, const pmf_instance *inst, int32_t n_inst, int64_t *flows_out,
                    int32_t *status_out) {
    if (!h || n_inst < 0 || (n_inst > 0 && (!inst || !flows_out))) return PMF_EINVAL;
    for (int i = 0; i < n_inst; ++i) {
        const int rc = check_instance(inst[i]);
        if (rc != PMF_OK) return rc;
    }
    h->solved = false;
    h->n_inst = 0;
    if (n_inst == 0) return PMF_OK;
    drop_graph(h);
    const Layout Lo = plan(inst, n_inst, h->opt);
    int rc = ensure_arena(h, Lo.total);
    if (rc != PMF_OK) return rc;
    char *A = h->arena;
    int tw, th;
    tile_dims(h->opt, &tw, &th);

    std::vector<InstDesc> desc(n_inst);
    std::vector<InstState> st(n_inst);
    std::vector<int32_t> tslot(Lo.ntiles), tlocal(Lo.ntiles);
    int64_t lam_base = 0;
    h->W.assign(n_inst, 0);
    h->H.assign(n_inst, 0);
    h->L.assign(n_inst, 0);
    h->masks_off.assign(n_inst, 0);
    for (int i = 0; i < n_inst; ++i) {
        const pmf_instance &I = inst[i];
        InstDesc &D = desc[i];
        std::memset(&D, 0, sizeof(D));
        D.W = I.W;
        D.H = I.H;
        D.K = I.K;
        D.n = I.W * I.H;
        D.tiles_x = Lo.tiles_x[i];
        D.tiles_y = Lo.tiles_y[i];
        D.ntiles = D.tiles_x * D.tiles_y;
        D.tile0 = Lo.tile0[i];
        D.L = I.L;
        D.slot_id = i;
        D.lambdas = I.lambdas;
        D.nlink = I.nlink;
        D.cap_src = I.cap_src;
        D.cap_snk0 = I.cap_snk0;
        D.slope = I.snk_slope;
        D.seed = I.seed;
        D.r = (int32_t *)(A + Lo.r[i]);
        D.e = (int32_t *)(A + Lo.e[i]);
        D.rt = (int32_t *)(A + Lo.rt[i]);
        D.h = (int32_t *)(A + Lo.h[i]);
        D.inbox = (int32_t *)(A + Lo.inbox[i]);
        D.rmask = (uint16_t *)(A + Lo.rmask[i]);
        D.masks = (uint8_t *)(A + Lo.masks[i]);
        D.flows = flows_out + lam_base;
        D.status = status_out ? status_out + i : nullptr;
        lam_base += I.L;
        std::memset(&st[i], 0, sizeof(InstState));
        st[i].phase = kInit;
        for (int t = 0; t < D.ntiles; ++t) {
            tslot[D.tile0 + t] = i;
            tlocal[D.tile0 + t] = t;
        }
        h->W[i] = I.W;
        h->H[i] = I.H;
        h->L[i] = I.L;
        h->masks_off[i] = Lo.masks[i];
    }
    hipStream_t s = h->stream;
    bool ok = true;
    ok &= hipMemcpyAsync(A + Lo.desc, desc.data(), sizeof(InstDesc) * n_inst, hipMemcpyHostToDevice, s) == hipSuccess;
    ok &= hipMemcpyAsync(A + Lo.st, st.data(), sizeof(InstState) * n_inst, hipMemcpyHostToDevice, s) == hipSuccess;
    ok &= hipMemcpyAsync(A + Lo.tile_slot, tslot.data(), 4 * (size_t)Lo.ntiles, hipMemcpyHostToDevice, s) == hipSuccess;
    ok &= hipMemcpyAsync(A + Lo.tile_local, tlocal.data(), 4 * (size_t)Lo.ntiles, hipMemcpyHostToDevice, s) == hipSuccess;
    ok &= hipMemsetAsync(A + Lo.ctl, 0, 64, s) == hipSuccess;
    if (!ok) return PMF_EDEVICE;

    StepParams P;
    std::memset(&P, 0, sizeof(P));
    P.desc = (InstDesc *)(A + Lo.desc);
    P.st = (InstState *)(A + Lo.st);
    P.tile_slot = (const int32_t *)(A + Lo.tile_slot);
    P.tile_local = (const int32_t *)(A + Lo.tile_local);
    P.tile_act = (uint32_t *)(A + Lo.tile_act);
    P.tile_chg = (uint8_t *)(A + Lo.tile_chg);
    P.tile_cnt = (int32_t *)(A + Lo.tile_cnt);
    P.arrive = (uint32_t *)(A + Lo.ctl);
    P.ndone = (int32_t *)(A + Lo.ctl + 4);
    P.counters = nullptr;
    P.ntiles = Lo.ntiles;
    P.per_xcd = (Lo.ntiles + 7) / 8;
    P.nslots = n_inst;
    P.inner_iters = h->opt.inner_iters;
    P.sweeps_per_relabel = h->opt.sweeps_per_relabel;
    P.local_bfs_iters = h->opt.local_bfs_iters;
    P.max_steps = h->opt.max_supersteps;

    const int S = h->opt.steps_per_sync;
    if (h->opt.use_graph) {
        hipGraph_t g = nullptr;
        ok = hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
        for (int i = 0; ok && i < S; ++i) ok = launch_superstep(P, tw, h->capture) == 0;
        const bool ended = hipStreamEndCapture(h->capture, &g) == hipSuccess;
        ok = ok && ended && hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (!ok) {
            (void)hipGetLastError();
            drop_graph(h);
            return PMF_EDEVICE;
        }
    }
    std::memset(&h->stats, 0, sizeof(h->stats));
    h->stats.device_bytes = (int64_t)h->arena_bytes;
    // Every instance ends within max_supersteps supersteps (device watchdog),
    // so this loop is bounded; the extra margin covers the final transitions.
    const int64_t max_rounds = h->opt.max_supersteps / S + 4;
    int64_t rounds = 0;
    for (;;) {
        if (h->graph) {
            if (hipGraphLaunch(h->graph, s) != hipSuccess) return PMF_EDEVICE;
        } else {
            for (int i = 0; i < S; ++i)
                if (launch_superstep(P, tw, s) != 0) return PMF_EDEVICE;
        }
        h->stats.supersteps += S;
        if (hipMemcpyAsync(h->pinned, P.ndone, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return PMF_EDEVICE;
        if (hipStreamSynchronize(s) != hipSuccess) return PMF_EDEVICE;
        h->stats.host_syncs += 1;
        if (*(volatile int32_t *)h->pinned >= n_inst) break;
        if (++rounds > max_rounds) return PMF_ETIMEOUT;
    }
    h->final_state.resize(n_inst);
    if (hipMemcpyAsync(h->final_state.data(), P.st, sizeof(InstState) * n_inst, hipMemcpyDeviceToHost, s) != hipSuccess)
        return PMF_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return PMF_EDEVICE;
    for (const InstState &x : h->final_state) {
        h->stats.sweep_visits += x.sweeps;
        h->stats.global_relabels += x.relabels;
        h->stats.bfs_passes += x.passes;
    }
    h->n_inst = n_inst;
    h->solved = true;
    return PMF_OK;
}

int pmf_extract_cut(pmf_handle *h, int32_t inst, int32_t lambda_idx, uint8_t *mask_out) {
    if (!h || !mask_out) return PMF_EINVAL;
    if (!h->solved) return PMF_ENOTSOLVED;
    if (inst < 0 || inst >= h->n_inst) return PMF_ERANGE;
    if (lambda_idx < 0 || lambda_idx >= h->L[inst]) return PMF_ERANGE;
    if (h->final_state[inst].k <= lambda_idx) return PMF_ENOTSOLVED;
    const size_t px = (size_t)h->W[inst] * h->H[inst];
    const char *src = h->arena + h->masks_off[inst] + (size_t)lambda_idx * px;
    if (hipMemcpyAsync(mask_out, src, px, hipMemcpyDeviceToDevice, h->stream) != hipSuccess) return PMF_EDEVICE;
    return PMF_OK;
}

int pmf_get_stats(pmf_handle *h, pmf_stats *out) {
    if (!h || !out) return PMF_EINVAL;
    *out = h->stats;
    return PMF_OK;
}

int pmf_destroy(pmf_handle *h) {
    if (!h) return PMF_EINVAL;
    (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    if (h->own_arena && h->arena) (void)hipFree(h->arena);
    if (h->pinned) (void)hipHostFree(h->pinned);
    if (h->capture) (void)hipStreamDestroy(h->capture);
    delete h;
    return PMF_OK;
}

}  // extern "C"
