#!/usr/bin/env python3
"""Throughput benchmark: exact max-flow solves/s on 500x375 4-connected grids.

One *step* solves one batch of the headline workload on the GPU through the C
ABI: 25 seeds (7x7 squares on a 5x5 lattice) of one synthetic 500x375 image,
each with the 20-point lambda schedule 1..2000, i.e. 500 (seed, lambda)
solves, packed into one call (warm-started chains).  Inputs are resident in
HBM before timing starts.  The same run also reports

* the same step with its transfers: inputs uploaded from pinned host memory,
  flows and the nested masks (one byte per pixel per seed) downloaded,
* the roofline of the tile-work kernels, from a solve in the library's timing
  mode (HIP events around every launch on the solver's stream, pixel visits
  counted per launch) with the algorithmic bytes per pixel visit of the
  method's state, next to a plain device-to-device copy of 1 GiB,
* the plain form: the same 25 chains solved one instance per call,
* the 8-connected variant of the same workload,
* the uneven workload: 256 images of 64..640 x 64..480, mixed connectivity,
  1..16 seeds, 10..30 lambdas each (about 42 000 solves in one call),
* all breakpoints of one seed over lambda in 1..2000 (integer change points,
  then every real breakpoint),
* the serving loop under Poisson arrivals at 50, 200 and 800 requests/s,
* the CPU oracle on every one of the 500 solves (host cores, one solve per
  thread), which also verifies every GPU flow and mask bit for bit,

and prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "exact max-flow solves/s (500×375 4-conn) batched vs plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
KINDS = ("sweep", "relabel", "cut", "init", "orient", "init_x", "cut_x")
# worker threads of the oracle pools: one GPU's share of the host's cores
HOST_SHARE = 16


def bytes_per_px(K: int, tw: int = 32, th: int = 32) -> dict:
    """Algorithmic bytes per pixel visit of each kind of tile work, counted on
    the method's per-pixel state (K residuals, excess, height, sink residual:
    (K + 3) int32 words):
    sweep: the state read and written once, the tile's halo heights, and the
    cross-tile pushes (one 4-byte word per border pixel and arc leaving the
    tile, written by the sender and read by the owner);
    relabel pass: the K residuals and the sink residual read, the label
    written ((K + 1) * 4 + 4); cut pass: the same reads and one mask byte
    ((K + 1) * 4 + 1); init: n-links, source, sink and slope planes and the
    seed byte read, the state written; orientation count: the terminal inputs
    read; exchanged init: also the reverse n-links; exchanged cut: a cut pass."""
    state = (K + 3) * 4
    halo = (2 * (tw + th) + 4) / (tw * th) * 4
    inbox = (2 if K == 4 else 6) * (tw + th) / (tw * th) * 8
    init = K * 4 + 13 + state
    return {"sweep": round(2 * state + halo + inbox, 3), "relabel": (K + 1) * 4 + 4, "cut": (K + 1) * 4 + 1,
            "init": init, "orient": 13, "init_x": init + K * 4, "cut_x": (K + 1) * 4 + 1}


def impl_bytes_per_px(K: int) -> dict:
    """What this implementation moves per pixel visit (its passes read a
    2-byte residual-bit word instead of the K + 1 residuals)."""
    init = K * 4 + 13 + K * 4 + 12 + 2
    return {"sweep": 2 * (K + 3) * 4 + 2, "relabel": 2 + 4 + 4, "cut": 2 + 1 + 1, "init": init,
            "orient": 13, "init_x": init + K * 4, "cut_x": 4 + 2 + 4 + 4 + 1}


def kind_bytes(px: list, b: dict) -> float:
    return float(sum(px[i] * b[k] for i, k in enumerate(KINDS)))


def stat_bytes(st: dict, b: dict) -> float:
    return float(sum(st["px_" + k] * b[k] for k in KINDS))


def gpu_masks(solver, insts):
    out = []
    for i, inst in enumerate(insts):
        out.append(np.stack([solver.extract_cut(i, k).cpu().numpy().astype(bool) for k in range(inst.L)]))
    return out


def host_info() -> dict:
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "cpus_available": avail}


def oracle_all(insts, threads: int):
    """Every (instance, lambda) solve of the batch by the oracle (cold, one
    single-threaded solve per task) on a thread pool; returns results and wall time."""
    from oracle import oracle as O
    O.build()
    tasks = [(inst, int(inst.lambdas[k])) for inst in insts for k in range(inst.L)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda t: O.fifo_pr(t[0], t[1]), tasks))
    return res, time.perf_counter() - t0


def verify_all(insts, flows, masks, results):
    """Flows and masks of every solve against the oracle, bit for bit."""
    bad, j = [], 0
    for i, inst in enumerate(insts):
        for k in range(inst.L):
            f, m = results[j]
            if int(flows[j]) != f or not (masks[i][k] == m).all():
                bad.append((i, k))
            j += 1
    return bad


def roofline(dev, overrides: dict, K: int, pmf, torch, split: bool = True) -> dict:
    """Timing-mode solve: HIP events around every tile-work launch (and every
    persistent launch) on the solver's stream, no host round trip between the
    supersteps of a poll, pixel visits counted per launch kind."""
    ts = pmf.Solver(timing=1, **overrides)
    ts.solve(dev)
    torch.cuda.synchronize()
    st = ts.stats()
    ts.close()
    tw = int(overrides.get("tile_w", 32) or 32)
    b = bytes_per_px(K, tw, 1024 // tw)
    bi = impl_bytes_per_px(K)
    kpx = st["kernel_px"]
    kernels = {}
    # timing mode launches the tile-work kernel under the symbol k_step<..., true> (same code)
    step_name = "k_step<%d, %d, %d, %s, true>" % (K, tw, 1024 // tw, "true" if overrides.get("gap") else "false")
    if st["work_launches"]:
        n = st["work_launches"]
        byt = kind_bytes(kpx[:7], b)
        kernels[step_name] = {"launches": n, "avg_launch_us": round(st["work_ns"] / n / 1e3, 3),
                              "alg_bytes_per_launch": int(byt / n), "total_ms": round(st["work_ns"] / 1e6, 3),
                              "achieved_GBs": round(byt / max(st["work_ns"], 1), 1),
                              "impl_bytes_per_launch": int(kind_bytes(kpx[:7], bi) / n),
                              "px_visits": dict(zip(KINDS, kpx[:7]))}
    pname = "k_persist<%d, %d, %d>" % (tw, 1024 // tw, K)
    if st["persist_launches"]:
        n = st["persist_launches"]
        byt = kind_bytes(kpx[8:15], b)
        kernels[pname] = {"launches": n, "avg_launch_us": round(st["persist_ns"] / n / 1e3, 3),
                          "supersteps": st["persist_supersteps"],
                          "alg_bytes_per_launch": int(byt / n), "total_ms": round(st["persist_ns"] / 1e6, 3),
                          "achieved_GBs": round(byt / max(st["persist_ns"], 1), 1),
                          "px_visits": dict(zip(KINDS, kpx[8:15]))}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    d = kernels[dom]
    achieved = d["alg_bytes_per_launch"] / (d["avg_launch_us"] * 1e-6) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
           "avg_launch_us": d["avg_launch_us"], "alg_bytes_per_launch": d["alg_bytes_per_launch"],
           "launches": d["launches"], "bytes_per_px": b, "impl_bytes_per_px": bi, "kernels": kernels,
           "supersteps": st["supersteps"], "device_ms": round(st["device_ns"] / 1e6, 3)}
    if not split:
        return out
    # timing mode 2: sweeps and passes as separate launches, each kind timed
    # apart (its own kernel start and end), for the sweep-only bandwidth
    sp = pmf.Solver(timing=2, **dict(overrides, persist_tiles=0))
    sp.solve(dev)
    torch.cuda.synchronize()
    ss = sp.stats()
    sp.close()
    spx = ss["kernel_px"][:7]
    sweep_b = spx[0] * b["sweep"]
    pass_b = kind_bytes(spx, b) - sweep_b
    tot = max(ss["sweep_ns"] + ss["pass_ns"] + ss["control_ns"], 1)
    out["split"] = {"sweep_GBs": round(sweep_b / max(ss["sweep_ns"], 1), 1),
                    "sweep_frac": round(sweep_b / max(ss["sweep_ns"], 1) / HBM_PEAK_GBS, 4),
                    "pass_GBs": round(pass_b / max(ss["pass_ns"], 1), 1),
                    "sweep_ms": round(ss["sweep_ns"] / 1e6, 3), "pass_ms": round(ss["pass_ns"] / 1e6, 3),
                    "control_ms": round(ss["control_ns"] / 1e6, 3),
                    "sweep_share": round(ss["sweep_ns"] / tot, 3), "pass_share": round(ss["pass_ns"] / tot, 3)}
    return out


def attach_profile(roof: dict, path: str) -> None:
    """The committed rocprofv3 summary of the dominant kernel: its average
    duration (kernel trace) and HBM traffic (FETCH_SIZE / WRITE_SIZE scaled by
    a 1 GiB copy), used while it still describes the current kernel sources."""
    from paper_1509_06004_amd import rocprof_summary
    prof = rocprof_summary.read_summary(path)
    if not prof:
        return
    current = prof.get("kernel_source_sha256") == rocprof_summary.source_hash()
    kname = roof["kernel"].replace(" ", "")
    info = {"file": os.path.relpath(path, ROOT), "current_sources": current}
    if "stats_avg_us" in prof and kname in prof.get("stats_kernel", "").replace(" ", ""):
        avg = float(prof["stats_avg_us"])
        info["avg_launch_us"] = avg
        info["achieved_at_profile_avg_GBs"] = round(roof["alg_bytes_per_launch"] / (avg * 1e-6) / 1e9, 1)
        info["event_over_profile"] = round(roof["avg_launch_us"] / avg, 3)
    if current and "traffic_bytes_per_launch" in prof and kname in prof.get("traffic_kernel", "").replace(" ", ""):
        roof["traffic"] = float(prof["traffic_bytes_per_launch"])
        info["traffic_over_alg"] = round(roof["traffic"] / max(roof["alg_bytes_per_launch"], 1), 3)
    roof["profile"] = info


def copy_bandwidth(torch) -> dict:
    """Attainable bandwidth on this device: a 1 GiB device-to-device copy
    (reads 1 GiB, writes 1 GiB), best of 5, timed with HIP events."""
    src = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) * 1e-3)
    del src, dst
    gbs = 2 * (1 << 30) / best / 1e9
    return {"bytes_moved": 2 * (1 << 30), "ms": round(best * 1e3, 3), "GBs": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def with_transfers(insts, pmf, torch, solver, steps: int) -> dict:
    """Steps that include the transfers: inputs copied from pinned host memory
    to fresh device buffers, the batch solved, flows and the nested masks
    (pmf_extract_levels: one byte per pixel per seed) copied back."""
    host = {}
    for inst in insts:
        for a in (inst.nlink, inst.cap_src, inst.cap_snk0, inst.snk_slope, inst.seed, inst.lambdas):
            if id(a) not in host:
                host[id(a)] = torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
    h2d = sum(t.numel() * t.element_size() for t in host.values())
    out_fl = torch.empty(sum(i.L for i in insts), dtype=torch.int64).pin_memory()
    out_lv = [torch.empty((i.H, i.W), dtype=torch.uint8).pin_memory() for i in insts]
    d2h = out_fl.numel() * 8 + sum(t.numel() for t in out_lv)
    times = []
    for s in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dev_arr = {k: t.to("cuda", non_blocking=True) for k, t in host.items()}
        dev = [pmf.DeviceInstance(i.W, i.H, i.K, dev_arr[id(i.nlink)], dev_arr[id(i.cap_src)],
                                  dev_arr[id(i.cap_snk0)], dev_arr[id(i.snk_slope)], dev_arr[id(i.seed)],
                                  dev_arr[id(i.lambdas)]) for i in insts]
        flows, status = solver.solve(dev)
        lv = []
        for i, d in enumerate(dev):
            t = torch.empty((d.H, d.W), dtype=torch.uint8, device="cuda")
            rc = pmf.pmf_extract_levels(solver.handle, i, int(t.data_ptr()))
            if rc != pmf.PMF_OK:
                raise pmf.PmfError(rc, "pmf_extract_levels")
            lv.append(t)
        out_fl.copy_(flows, non_blocking=True)
        for o, t in zip(out_lv, lv):
            o.copy_(t, non_blocking=True)
        torch.cuda.synchronize()
        if s:
            times.append(time.perf_counter() - t0)
    n = sum(i.L for i in insts)
    return {"value": round(n * len(times) / sum(times), 2), "unit": "solves/s",
            "ms_per_step": round(sum(times) / len(times) * 1e3, 2), "h2d_bytes": int(h2d), "d2h_bytes": int(d2h),
            "what": "per step: inputs from pinned host memory to the device, the batched solve, flows and the "
                    "nested masks (one byte per pixel per seed) back to pinned host memory"}


def run_serving(qps: float, seconds: float, warmup: float, templates: int, inflight: int, log,
                chunk: int = 0, persist: dict = None) -> dict:
    """The serving workload: Poisson requests (one image, 1..32 seeds, 10..30
    lambdas each) served by the continuous-batching loop on one session."""
    from paper_1509_06004_amd import workload
    from paper_1509_06004_amd.serve import PmfBackend, Server
    arrivals, pick, pool = workload.config4_stream(qps, seconds, warmup, templates=templates)
    be = PmfBackend(max_slots=4096, supersteps=16, lambda_chunk=chunk, **(persist or {}))
    srv = Server(be, max_inflight_instances=inflight)
    rep = srv.run(arrivals, lambda i: pool[pick[i]], duration_s=seconds, warmup_s=warmup, qps=qps)
    be.close()
    out = rep.summary()
    out["workload"] = ("Poisson arrivals; request = one synthetic image 128x96..640x480 (K 4 or 8) with "
                       "1..32 seeds x 10..30 lambdas in [1, 5000], drawn from %d generated images" % templates)
    out["max_inflight_instances"] = inflight
    out["lambda_chunk"] = chunk
    out["seconds"] = seconds
    out["warmup_s"] = warmup
    log("serving qps %g: %s" % (qps, json.dumps({k: v for k, v in out.items() if k != "workload"})))
    return out


def leg_options(insts, log, cli: dict) -> dict:
    """Options for a leg of the bench: the tuner cache's entry for that
    workload class on this device if there is one, else library defaults;
    command-line overrides on top."""
    _, opts, _ = tuned_options(insts, log)
    out = dict(opts or {})
    out.update(cli)
    if "tile_w" in out:
        out["tile_h"] = 1024 // out["tile_w"]
    return out


def tuned_options(insts, log) -> tuple:
    """Knob values of the committed tuner cache for this workload class and
    device, if present."""
    from paper_1509_06004_amd import tune as T
    import torch
    key = T.workload_key(insts, torch.cuda.get_device_name(0))
    cache = T.load_cache(T.PACKAGE_CACHE)
    if key in cache:
        log("tuner cache hit: %s" % key)
        return key, dict(cache[key]["options"]), cache[key]
    log("tuner cache has no entry for %s" % key)
    return key, None, None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--opt", action="append", default=[], metavar="NAME=VALUE",
                    help="solver option override (repeatable), e.g. --opt persist_tiles=0")
    ap.add_argument("--defaults", action="store_true", help="ignore the tuner cache; library defaults")
    ap.add_argument("--tune-8conn", action="store_true",
                    help="autotune the 8-connected variant of the workload first and store the result in the "
                         "package's tuner cache (its bench leg then uses it)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the speed knobs on this workload first and store the result in the "
                         "package's tuner cache (results must not change)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-8conn", action="store_true")
    ap.add_argument("--no-config3", action="store_true")
    ap.add_argument("--no-transfers", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-breakpoints", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the split-timing solve (for profiled runs: the timed tile-work symbol then "
                         "covers exactly the launches of the fused timing solve)")
    ap.add_argument("--serve-qps", type=float, action="append", default=[],
                    help="serving rates (default 50, 200, 800)")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-templates", type=int, default=24)
    ap.add_argument("--serve-inflight", type=int, default=768)
    ap.add_argument("--serve-chunk", type=int, default=0,
                    help="lambdas per device instance in serving (0: whole schedules)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="finish with one 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: instances are independent, so more GPUs would each "
              "take their own share of the instances (a host router, no exchange between GPUs); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1509_06004_amd import pmf, workload

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    insts = workload.config2(K=4)
    n_solves = sum(i.L for i in insts)
    dev = pmf.to_device(insts)

    def tune_and_store(tinsts, tdev, what):
        # coordinate descent over the speed knobs on this workload; the result
        # goes to the package's tuner cache under the workload's class
        from paper_1509_06004_amd import tune as T
        t0 = time.perf_counter()
        res = T.tune(tdev, log=log)
        if res["rejected"]:
            raise SystemExit("autotuner found configurations with different results: %s" % res["rejected"])
        key = T.workload_key(tinsts, torch.cuda.get_device_name(0))
        cache = T.load_cache(T.PACKAGE_CACHE)
        cache[key] = {"options": res["options"], "seconds": res["seconds"], "trials": len(res["trials"]),
                      "confirmed": res["confirmed"], "tuned_on": what}
        T.save_cache(cache, T.PACKAGE_CACHE)
        return key, res, round(time.perf_counter() - t0, 1)

    if args.tune_8conn:
        insts8 = workload.config2(K=8)
        tune_and_store(insts8, pmf.to_device(insts8), "500x375 8-connected, 25 seeds x 20 lambdas")

    tuned = None
    overrides = {}
    if args.tune:
        key, res, secs = tune_and_store(insts, dev, "500x375 4-connected, 25 seeds x 20 lambdas")
        tuned = {"source": "tuned in this run", "key": key, "options": res["options"],
                 "tune_seconds": secs, "trials": len(res["trials"])}
        overrides = dict(res["options"])
    elif not args.defaults:
        key, opts, entry = tuned_options(insts, log)
        if opts is not None:
            overrides = opts
            from paper_1509_06004_amd import tune as T
            tuned = {"source": os.path.relpath(T.PACKAGE_CACHE, ROOT), "key": key, "options": opts}
    cli = {}
    for kv in args.opt:
        k, v = kv.split("=", 1)
        cli[k] = int(v)
    overrides.update(cli)
    if "tile_w" in overrides:
        overrides["tile_h"] = 1024 // overrides["tile_w"]

    def other(leg_insts):
        # the other legs use options tuned for their own workload class (or the defaults)
        return cli if args.defaults else leg_options(leg_insts, log, cli)

    solver = pmf.Solver(**overrides)
    torch.cuda.synchronize()
    log("workload: %d instances, %d solves; warmup %d; options %s" % (len(insts), n_solves, args.warmup, overrides))
    for _ in range(args.warmup):
        solver.solve(dev)
    torch.cuda.synchronize()

    times, dev_ns = [], 0
    flows = status = None
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for s in range(args.steps):
        t0 = time.perf_counter()
        flows, status = solver.solve(dev)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        dev_ns += solver.stats()["device_ns"]
        log("step %d: %.1f ms" % (s, times[-1] * 1e3))
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    value = n_solves * args.steps / total
    flows_np = flows.cpu().numpy()
    status_np = status.cpu().numpy()
    assert (status_np == 0).all(), status_np
    last = solver.stats()
    masks = gpu_masks(solver, insts)

    out = {"metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(total / args.steps * 1e3, 2),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic",
           "config": {"workload": "500x375 4-connected grid, 24-region synthetic image, 25 seeds "
                                  "(7x7, 5x5 lattice) x 20 geometric lambdas 1..2000 = 500 solves per "
                                  "step, one pmf_solve_batch call, inputs resident in HBM",
                      "options": {f: getattr(solver.options, f) for f, _ in pmf.Options._fields_
                                  if f not in ("max_supersteps", "mem_budget", "max_slots", "timing")}},
           "latency_ms": {"p50": round(float(np.percentile(times, 50)) * 1e3, 2),
                          "p99": round(float(np.percentile(times, 99)) * 1e3, 2),
                          "what": "per batched step of 500 solves"},
           "device_time_frac": round(dev_ns * 1e-9 / sum(times), 3),
           "per_step": {"supersteps": last["supersteps"], "persist_supersteps": last["persist_supersteps"],
                        "host_syncs": last["host_syncs"],
                        "px_visits": {k: last["px_" + k] for k in KINDS},
                        "alg_GB": round(stat_bytes(last, bytes_per_px(4)) / 1e9, 3)},
           "autotuned": tuned}

    if not args.no_transfers:
        out["with_transfers"] = with_transfers(insts, pmf, torch, solver, max(3, args.steps // 4))
        log("with transfers: %s" % out["with_transfers"])

    if not args.no_roofline:
        roof = roofline(dev, overrides, 4, pmf, torch, split=not args.no_split)
        attach_profile(roof, os.path.join(ROOT, "profiles", "k_step_500x375_4conn.txt"))
        if not args.no_copy:
            roof["copy"] = copy_bandwidth(torch)
        out["roofline"] = roof
        log("roofline: %s" % json.dumps({k: v for k, v in roof.items() if k != "kernels"}))

    # plain: one instance (one seed's 20-lambda warm chain) per call, same
    # kernels, same GPU, same run
    if not args.no_plain:
        # library defaults (knobs tuned for the packed batch, e.g. the
        # persistent launch, can slow a lone chain down)
        psolver = pmf.Solver(lambda_chunk=max(i.L for i in insts))
        psolver.solve([dev[0]])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain_lat = []
        for d in dev:
            t1 = time.perf_counter()
            psolver.solve([d])
            torch.cuda.synchronize()
            plain_lat.append(time.perf_counter() - t1)
        pt = time.perf_counter() - t0
        plain = n_solves / pt
        psolver.close()
        out["plain"] = {"value": round(plain, 2), "unit": "solves/s",
                        "form": "one instance (one seed's 20-lambda warm chain) per pmf_solve_batch call, "
                                "library default options",
                        "chain_latency_ms": {"p50": round(float(np.percentile(plain_lat, 50)) * 1e3, 2),
                                             "p99": round(float(np.percentile(plain_lat, 99)) * 1e3, 2)}}
        out["batched_over_plain"] = round(value / plain, 2)
        log("plain %.1f solves/s" % plain)

    if not args.no_8conn:
        insts8 = workload.config2(K=8)
        dev8 = pmf.to_device(insts8)
        o8 = other(insts8)
        solver8 = pmf.Solver(**o8)
        solver8.solve(dev8)
        torch.cuda.synchronize()
        t8 = []
        for _ in range(3):
            t0 = time.perf_counter()
            solver8.solve(dev8)
            torch.cuda.synchronize()
            t8.append(time.perf_counter() - t0)
        st8 = solver8.stats()
        solver8.close()
        c8 = {"value": round(n_solves * len(t8) / sum(t8), 2), "unit": "solves/s",
              "workload": "same, 8-connected (diagonals / sqrt 2)", "options": o8 or "library defaults",
              "alg_GB_per_step": round(stat_bytes(st8, bytes_per_px(8)) / 1e9, 3)}
        if not args.no_roofline:
            r8 = roofline(dev8, o8, 8, pmf, torch, split=False)
            c8["roofline"] = {k: r8[k] for k in ("kernel", "achieved", "frac", "avg_launch_us",
                                                 "alg_bytes_per_launch", "launches")}
        out["config_8conn"] = c8
        del dev8
        log("8-conn %s" % json.dumps(c8))

    if not args.no_config3:
        t0 = time.perf_counter()
        insts3 = workload.config3()
        gen = time.perf_counter() - t0
        dev3 = pmf.to_device(insts3)
        n3 = sum(i.L for i in insts3)
        o3 = other(insts3)
        s3 = pmf.Solver(**o3)
        s3.solve(dev3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f3, st3 = s3.solve(dev3)
        torch.cuda.synchronize()
        t3 = time.perf_counter() - t0
        ok3 = bool((st3.cpu().numpy() == 0).all())
        stats3 = s3.stats()
        b4, b8 = bytes_per_px(4), bytes_per_px(8)
        frac8 = sum(i.W * i.H * i.L for i in insts3 if i.K == 8) / sum(i.W * i.H * i.L for i in insts3)
        alg3 = (1 - frac8) * stat_bytes(stats3, b4) + frac8 * stat_bytes(stats3, b8)
        s3.close()
        out["config3"] = {"value": round(n3 / t3, 2), "unit": "solves/s", "solves": n3, "instances": len(insts3),
                          "ms": round(t3 * 1e3, 2), "all_ok": ok3, "generate_s": round(gen, 1),
                          "options": o3 or "library defaults",
                          "alg_GB": round(alg3 / 1e9, 3),
                          "alg_GBs_over_device_time": round(alg3 / max(stats3["device_ns"], 1), 1),
                          "workload": "256 images 64..640 x 64..480, K 4 or 8, 8..48 regions, 1..16 seeds "
                                      "(7x7), 10..30 log-uniform lambdas in [1, 5000], one pmf_solve_batch call"}
        del dev3
        log("config3: %s" % json.dumps(out["config3"]))

    if not args.no_breakpoints:
        # the second workload on the same kernels: every lambda in 1..2000 at
        # which the minimal source set of one seed's instance changes
        bsolver = pmf.Solver(**cli)
        binst = pmf.to_device([insts[0]])[0]
        pmf.pmf_parametric(bsolver.handle, binst, 1, 2000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bps, bfl, _ = pmf.pmf_parametric(bsolver.handle, binst, 1, 2000)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        pmf.pmf_breakpoints(bsolver.handle, binst, 1, 2000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rnum, rden, _, _, _ = pmf.pmf_breakpoints(bsolver.handle, binst, 1, 2000)
        torch.cuda.synchronize()
        tr = time.perf_counter() - t0
        bsolver.close()
        out["breakpoints"] = {"range": [1, 2000], "change_points": int(len(bps)), "ms": round(tb * 1e3, 2),
                              "workload": "seed 0 of the headline workload: all integer lambdas in 1..2000 at "
                                          "which S_min changes, F there and each pixel's exit lambda",
                              "real": {"breakpoints": int(len(rnum)),
                                       "largest_denominator": int(rden.max()) if len(rden) else 1,
                                       "ms": round(tr * 1e3, 2),
                                       "workload": "the same instance and range: every real breakpoint as a "
                                                   "fraction, the line of F on each piece, each pixel's exit piece"}}
        log("breakpoints: %d integer change points in %.1f ms, %d real breakpoints in %.1f ms"
            % (len(bps), tb * 1e3, len(rnum), tr * 1e3))

    if not args.no_serve:
        rates = args.serve_qps or [50.0, 200.0, 800.0]
        persist = {k: cli[k] for k in ("persist_tiles", "persist_wgs", "gap") if k in cli}
        out["serving"] = [run_serving(q, args.serve_seconds, args.serve_warmup, args.serve_templates,
                                      args.serve_inflight, log, args.serve_chunk, persist) for q in rates]
        sv = out["serving"][0]
        out["latency_ms"] = dict(sv["latency_ms"], what="serving: scheduled arrival to results on host, "
                                                         "%g requests/s" % sv["qps"])
        out["latency_ms_batched_step"] = {"p50": round(float(np.percentile(times, 50)) * 1e3, 2),
                                          "p99": round(float(np.percentile(times, 99)) * 1e3, 2)}
        out["served_over_plain"] = (round(max(s["solves_per_s"] for s in out["serving"]) / out["plain"]["value"], 2)
                                    if "plain" in out else None)

    if not args.no_cpu:
        threads = max(1, min(host_info()["cpus_available"], HOST_SHARE))
        res, wall = oracle_all(insts, threads)
        from oracle import oracle as O
        one = [(insts[i], int(insts[i].lambdas[k])) for i, k in ((0, 0), (6, 5), (12, 10), (18, 15), (24, 19))]
        t1 = time.perf_counter()
        for inst_, lam_ in one:
            O.fifo_pr(inst_, lam_)
        wall1 = time.perf_counter() - t1
        out["cpu_baseline"] = dict({"value": round(n_solves / wall, 2), "unit": "solves/s", "cores": threads,
                                    "kind": "oracle",
                                    "sample": "all %d (seed, lambda) solves of one step, each solved from "
                                              "scratch by FIFO push-relabel (int64), one per thread, %d threads "
                                              "(one GPU's share of the host)" % (n_solves, threads),
                                    "value_1core": round(len(one) / wall1, 2),
                                    "sample_1core": "%d solves spread over the schedule, one after another on "
                                                    "one core" % len(one)}, **host_info())
        log("cpu %.2f solves/s on %d threads" % (n_solves / wall, threads))
        bad = verify_all(insts, flows_np, masks, res)
        out["verified"] = {"oracle_mismatches": len(bad), "solves_compared": n_solves,
                           "what": "every flow and every mask of the last timed step against the oracle"}
        if bad:
            print(json.dumps(out))
            raise SystemExit("verification failed at %s" % bad[:10])
    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
