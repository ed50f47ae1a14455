#!/usr/bin/env python3
"""Throughput benchmark: exact max-flow solves/s on 500x375 4-connected grids.

One *step* solves one batch of the headline workload on the GPU through the C
ABI: 25 seeds (7x7 squares on a 5x5 lattice) of one synthetic 500x375 image,
each with the 20-point lambda schedule 1..2000, i.e. 500 (seed, lambda)
solves, packed into one call (warm-started chains).  Inputs are resident in
HBM before timing starts.  The same run also times

* the plain form: the same 25 chains solved one instance per call,
* the 8-connected variant of the same workload,
* the CPU oracle on a bounded sample of the same solves (host cores),

verifies a sample of the GPU results against the oracle (bit-exact flows and
masks) and all of them against the max-flow/min-cut certificate and nesting,
and prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "exact max-flow solves/s (500×375 4-conn) batched vs plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def bytes_per_px(K: int) -> dict:
    """Algorithmic bytes per pixel visit of each phase (the solver's own state):
    sweep: read + write r_k, e, rt, h (int32) + write the residual bit word;
    relabel pass: read bit word + read/write h; cut pass: bit word + mask r/w;
    init: read n-links and terminal inputs, write the whole state (exchanged:
    also the reverse n-links); orientation count: terminal inputs; exchanged
    cut: h, bit word, e, rt read, mask written."""
    init = K * 4 + 13 + K * 4 + 12 + 2
    return {"sweep": 2 * (K + 3) * 4 + 2, "relabel": 2 + 4 + 4, "cut": 2 + 1 + 1, "init": init,
            "orient": 13, "init_x": init + K * 4, "cut_x": 4 + 2 + 4 + 4 + 1}


def alg_bytes(st: dict, K: int) -> float:
    b = bytes_per_px(K)
    return (st["px_sweep"] * b["sweep"] + st["px_relabel"] * b["relabel"] + st["px_cut"] * b["cut"]
            + st["px_init"] * b["init"] + st["px_orient"] * b["orient"] + st["px_init_x"] * b["init_x"]
            + st["px_cut_x"] * b["cut_x"])


def add_stats(acc: dict, st: dict):
    for k, v in st.items():
        acc[k] = acc.get(k, 0) + v


def gpu_masks(solver, insts):
    out = []
    for i, inst in enumerate(insts):
        out.append(np.stack([solver.extract_cut(i, k).cpu().numpy().astype(bool) for k in range(inst.L)]))
    return out


def verify(insts, flows, masks, sample_pairs, oracle_results):
    """Bit-exact against the oracle on the sample; certificate + nesting on all."""
    from oracle import oracle as O
    off = np.cumsum([0] + [i.L for i in insts])
    bad = 0
    for (i, k), (f, m) in zip(sample_pairs, oracle_results):
        bad += int(flows[off[i] + k]) != f or not (masks[i][k] == m).all()
    cert = 0
    for i, inst in enumerate(insts):
        for k in range(inst.L):
            cert += O.cut_cost_c(inst, int(inst.lambdas[k]), masks[i][k]) != int(flows[off[i] + k])
            if k:
                cert += bool((masks[i][k] & ~masks[i][k - 1]).any())
    return bad, cert


def cpu_baseline(insts, n_sample: int, threads: int):
    """The oracle (cold, one single-threaded solve per task) on a thread pool."""
    from oracle import oracle as O
    O.build()
    pairs = []
    L = insts[0].L
    total = len(insts) * L
    for j in range(n_sample):
        idx = (j * total) // n_sample
        pairs.append((idx // L, idx % L))
    tasks = [(insts[i], int(insts[i].lambdas[k])) for i, k in pairs]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda t: O.fifo_pr(t[0], t[1]), tasks))
    wall = time.perf_counter() - t0
    return pairs, res, wall


def run_serving(qps: float, seconds: float, warmup: float, templates: int, inflight: int, log,
                chunk: int = 1) -> dict:
    """The serving workload: Poisson requests (one image, 1..32 seeds, 10..30
    lambdas each) served by the continuous-batching loop on one session."""
    from paper_1509_06004_amd import workload
    from paper_1509_06004_amd.serve import PmfBackend, Server
    arrivals, pick, pool = workload.config4_stream(qps, seconds, warmup, templates=templates)
    be = PmfBackend(max_slots=4096, supersteps=16, lambda_chunk=chunk)
    srv = Server(be, max_inflight_instances=inflight)
    rep = srv.run(arrivals, lambda i: pool[pick[i]], duration_s=seconds, warmup_s=warmup, qps=qps)
    be.close()
    out = rep.summary()
    out["workload"] = ("Poisson arrivals; request = one synthetic image 128x96..640x480 (K 4 or 8) with "
                       "1..32 seeds x 10..30 lambdas in [1, 5000], drawn from %d generated images" % templates)
    out["max_inflight_instances"] = inflight
    out["lambda_chunk"] = chunk
    out["warmup_s"] = warmup
    log("serving qps %g: %s" % (qps, json.dumps({k: v for k, v in out.items() if k != "workload"})))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tile-w", type=int, default=0)
    ap.add_argument("--inner-iters", type=int, default=0)
    ap.add_argument("--sweeps-per-relabel", type=int, default=0)
    ap.add_argument("--local-bfs-iters", type=int, default=0)
    ap.add_argument("--steps-per-sync", type=int, default=0)
    ap.add_argument("--lambda-chunk", type=int, default=0)
    ap.add_argument("--exchange-rounds", type=int, default=0)
    ap.add_argument("--tail-tiles", type=int, default=-1, help="0 disables the short-superstep settings")
    ap.add_argument("--tail-inner-iters", type=int, default=0)
    ap.add_argument("--tail-exchange-rounds", type=int, default=0)
    ap.add_argument("--relabel-passes", type=int, default=-1, help="0 runs every relabel to its fixed point")
    ap.add_argument("--orientation", type=int, default=-1,
                    help="s-t swap rule: 0 as given, 1 paper's rule, 2 inverse rule, 3 always")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the speed knobs on this workload before timing (results must not change)")
    ap.add_argument("--cpu-sample", type=int, default=48)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-8conn", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-breakpoints", action="store_true")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the split-timing solve (profiled runs: every k_step launch is then fused as in "
                         "the timed solves)")
    ap.add_argument("--serve-qps", type=float, default=50.0)
    ap.add_argument("--serve-seconds", type=float, default=8.0)
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-templates", type=int, default=12)
    ap.add_argument("--serve-inflight", type=int, default=768)
    ap.add_argument("--serve-chunk", type=int, default=0,
                    help="lambdas per device instance in serving (0: whole schedules)")
    ap.add_argument("--serve-full", action="store_true",
                    help="serving sweep at 50, 200 and 800 requests/s, 60 s each after 5 s warm-up")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="finish with one 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: instances are independent, so more GPUs would each "
              "run their own copy of this workload (see the sharding note in DESIGN.md); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1509_06004_amd import pmf, workload

    torch.cuda.set_device(0)
    overrides = {}
    if args.tile_w:
        overrides.update(tile_w=args.tile_w, tile_h=1024 // args.tile_w)
    for a, f in (("inner_iters", args.inner_iters), ("sweeps_per_relabel", args.sweeps_per_relabel),
                 ("local_bfs_iters", args.local_bfs_iters), ("steps_per_sync", args.steps_per_sync),
                 ("lambda_chunk", args.lambda_chunk), ("exchange_rounds", args.exchange_rounds),
                 ("tail_inner_iters", args.tail_inner_iters), ("tail_exchange_rounds", args.tail_exchange_rounds)):
        if f:
            overrides[a] = f
    if args.tail_tiles >= 0:
        overrides["tail_tiles"] = args.tail_tiles
    if args.relabel_passes >= 0:
        overrides["relabel_passes"] = args.relabel_passes
    if args.orientation >= 0:
        overrides["orientation"] = args.orientation

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    insts = workload.config2(K=4)
    n_solves = sum(i.L for i in insts)
    dev = pmf.to_device(insts)
    tuned = None
    if args.tune:
        from paper_1509_06004_amd import tune as T
        t0 = time.perf_counter()
        res = T.tune(dev, start=overrides or None, log=log)
        tuned = {"options": res["options"], "tune_seconds": round(time.perf_counter() - t0, 1),
                 "trials": len(res["trials"]), "rejected": len(res["rejected"])}
        if res["rejected"]:
            raise SystemExit("autotuner found configurations with different results: %s" % res["rejected"])
        overrides = dict(res["options"])
        overrides["tile_h"] = 1024 // overrides["tile_w"]
    solver = pmf.Solver(**overrides)
    torch.cuda.synchronize()
    log("workload: %d instances, %d solves; warmup %d" % (len(insts), n_solves, args.warmup))
    for _ in range(args.warmup):
        solver.solve(dev)
    torch.cuda.synchronize()

    times, acc = [], {}
    flows = status = None
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for s in range(args.steps):
        t0 = time.perf_counter()
        flows, status = solver.solve(dev)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        add_stats(acc, solver.stats())
        log("step %d: %.1f ms" % (s, times[-1] * 1e3))
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    value = n_solves * args.steps / total
    flows_np = flows.cpu().numpy()
    status_np = status.cpu().numpy()
    assert (status_np == 0).all(), status_np

    # roofline of the dominant kernel (k_step: the sweeps and the relabel / cut
    # / init passes of one superstep): one extra solve in the library's timing
    # mode, which brackets every launch with HIP events on the solver's stream,
    # and one in its split mode (sweeps and passes launched apart) for shares
    tsolver = pmf.Solver(timing=1, **overrides)
    tsolver.solve(dev)
    torch.cuda.synchronize()
    ts = tsolver.stats()
    tsolver.close()
    ss = None
    if not args.no_split:
        ssolver = pmf.Solver(timing=2, **overrides)
        ssolver.solve(dev)
        torch.cuda.synchronize()
        ss = ssolver.stats()
        ssolver.close()
    bpx = bytes_per_px(4)
    work_bytes = alg_bytes(ts, 4)
    n_work = max(ts["work_launches"], 1)
    per_launch_bytes = work_bytes / n_work
    avg_launch_s = ts["work_ns"] * 1e-9 / n_work
    achieved = per_launch_bytes / avg_launch_s / 1e9
    tw = solver.options.tile_w
    kname = "k_step<4, %d, %d>" % (tw, 1024 // tw)
    # HBM bytes per launch from the committed counter summary, while it still
    # describes the current kernel source
    from paper_1509_06004_amd import rocprof_summary
    prof = rocprof_summary.read_summary(os.path.join(ROOT, "profiles", "k_step_500x375_4conn_traffic.txt"))
    traffic = None
    if (prof.get("kernel_source_sha256") == rocprof_summary.source_hash()
            and "traffic_bytes_per_launch" in prof
            and kname.replace(" ", "") in prof.get("traffic_kernel", "").replace(" ", "")):
        traffic = float(prof["traffic_bytes_per_launch"])
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kname, "avg_launch_us": round(avg_launch_s * 1e6, 2),
            "alg_bytes_per_launch": int(per_launch_bytes), "launches": int(n_work),
            "bytes_per_px": bpx}
    if ss is not None:
        split_total = max(ss["sweep_ns"] + ss["pass_ns"] + ss["control_ns"], 1)
        roof["split"] = {"sweep_GBs": round(ss["px_sweep"] * bpx["sweep"] / max(ss["sweep_ns"], 1), 1),
                         "pass_GBs": round((alg_bytes(ss, 4) - ss["px_sweep"] * bpx["sweep"])
                                           / max(ss["pass_ns"], 1), 1),
                         "sweep_share": round(ss["sweep_ns"] / split_total, 3),
                         "pass_share": round(ss["pass_ns"] / split_total, 3),
                         "control_share": round(ss["control_ns"] / split_total, 3)}

    out = {"metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(total / args.steps * 1e3, 2),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic",
           "config": {"workload": "500x375 4-connected grid, 24-region synthetic image, 25 seeds "
                                  "(7x7, 5x5 lattice) x 20 geometric lambdas 1..2000 = 500 solves per "
                                  "step, one pmf_solve_batch call",
                      "options": {k: getattr(solver.options, k) for k in
                                  ("tile_w", "tile_h", "inner_iters", "sweeps_per_relabel",
                                   "local_bfs_iters", "exchange_rounds", "tail_tiles", "tail_inner_iters",
                                   "tail_exchange_rounds", "relabel_passes", "orientation", "steps_per_sync",
                                   "use_graph", "order",
                                   "lambda_chunk")}},
           "latency_ms": {"p50": round(float(np.percentile(times, 50)) * 1e3, 2),
                          "p99": round(float(np.percentile(times, 99)) * 1e3, 2),
                          "what": "per batched step of 500 solves"},
           "device_time_frac": round(acc["device_ns"] * 1e-9 / sum(times), 3),
           "autotuned": tuned,
           "roofline": roof}

    # plain: one instance (one seed's 20-lambda chain, warm-started, not split)
    # per call, same kernels, same GPU, same run
    if not args.no_plain:
        psolver = pmf.Solver(lambda_chunk=max(i.L for i in insts), **overrides)
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
                        "form": "one instance (one seed's 20-lambda warm chain) per pmf_solve_batch call",
                        "chain_latency_ms": {"p50": round(float(np.percentile(plain_lat, 50)) * 1e3, 2),
                                             "p99": round(float(np.percentile(plain_lat, 99)) * 1e3, 2)}}
        out["batched_over_plain"] = round(value / plain, 2)
        log("plain %.1f solves/s" % plain)

    masks = gpu_masks(solver, insts) if not args.no_verify else None

    if not args.no_8conn:
        insts8 = workload.config2(K=8)
        dev8 = pmf.to_device(insts8)
        solver.solve(dev8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.solve(dev8)
        torch.cuda.synchronize()
        t8 = time.perf_counter() - t0
        st8 = solver.stats()
        out["config_8conn"] = {"value": round(n_solves / t8, 2), "unit": "solves/s",
                               "workload": "same, 8-connected (diagonals / sqrt 2)",
                               "achieved_GBs": round(alg_bytes(st8, 8) / (st8["device_ns"] * 1e-9) / 1e9, 1)}
        del dev8
        log("8-conn %.1f solves/s" % (n_solves / t8))

    if not args.no_breakpoints:
        # the second workload on the same kernels: every lambda in 1..2000 at
        # which the minimal source set of one seed's instance changes
        bsolver = pmf.Solver(**overrides)
        binst = pmf.to_device([insts[0]])[0]
        pmf.pmf_parametric(bsolver.handle, binst, 1, 2000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bps, bfl, _ = pmf.pmf_parametric(bsolver.handle, binst, 1, 2000)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        bsolver.close()
        out["breakpoints"] = {"range": [1, 2000], "change_points": int(len(bps)), "ms": round(tb * 1e3, 2),
                              "workload": "seed 0 of the headline workload: all integer lambdas in 1..2000 at "
                                          "which S_min changes, F there and each pixel's exit lambda"}
        log("breakpoints: %d in %.1f ms" % (len(bps), tb * 1e3))

    if not args.no_serve:
        if args.serve_full:
            out["serving"] = [run_serving(q, 60.0, 5.0, 24, args.serve_inflight, log, args.serve_chunk)
                              for q in (50.0, 200.0, 800.0)]
        else:
            out["serving"] = run_serving(args.serve_qps, args.serve_seconds, args.serve_warmup,
                                         args.serve_templates, args.serve_inflight, log, args.serve_chunk)
        sv = out["serving"] if isinstance(out["serving"], dict) else out["serving"][0]
        out["latency_ms"] = dict(sv["latency_ms"], what="serving: scheduled arrival to results on host, "
                                                         "%g requests/s" % sv["qps"])
        out["latency_ms_batched_step"] = {"p50": round(float(np.percentile(times, 50)) * 1e3, 2),
                                          "p99": round(float(np.percentile(times, 99)) * 1e3, 2)}

    if not args.no_cpu:
        threads = min(os.cpu_count() or 1, 16)
        pairs, res, wall = cpu_baseline(insts, args.cpu_sample, threads)
        # the same oracle on one core: every 6th solve of the sample, one after another
        from oracle import oracle as O
        one = [(insts[i], int(insts[i].lambdas[k])) for i, k in pairs[::6]]
        t1 = time.perf_counter()
        for inst_, lam_ in one:
            O.fifo_pr(inst_, lam_)
        wall1 = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(len(pairs) / wall, 2), "unit": "solves/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "%d of the %d (seed, lambda) solves, evenly spaced, each solved "
                                         "from scratch by FIFO push-relabel (int64), one per thread"
                                         % (len(pairs), n_solves),
                               "value_1core": round(len(one) / wall1, 2),
                               "sample_1core": "every 6th of those (%d solves), one core" % len(one)}
        log("cpu %.2f solves/s on %d threads" % (len(pairs) / wall, threads))
        if masks is not None:
            bad, cert = verify(insts, flows_np, masks, pairs, res)
            out["verified"] = {"oracle_sample_mismatches": bad, "certificate_or_nesting_failures": cert,
                               "sampled": len(pairs), "checked_by_certificate": n_solves}
            if bad or cert:
                print(json.dumps(out))
                raise SystemExit("verification failed")
    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
