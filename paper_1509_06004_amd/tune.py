"""Autotuner for the solver's speed knobs.

The knobs change speed, never results: tile shape, push/relabel iterations per
tile visit, sweeps between global relabels, the bound on relaxation rounds per
tile visit, halo exchange rounds per pass, the settings of short (latency
bound) supersteps, the orientation (s-t swap) rule, packing order (FIFO or
largest-first), the lambda chunk (how the schedule of each instance is cut
into concurrently solved pieces), the gap heuristic, and when and how wide
the persistent (cooperative) superstep launch runs.  The
tuner times solves of a calibration set on the device by coordinate descent
from the defaults and keeps the fastest point.  Every point's flows and masks
must equal those of the starting point bit for bit; a point that differs is
rejected and reported (it would be a solver bug).

Results are cached in a JSON file keyed by the workload class (size buckets,
connectivity, schedule length) and the device name.
"""

from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence

from . import pmf

KNOBS = ("tile_w", "inner_iters", "sweeps_per_relabel", "local_bfs_iters", "exchange_rounds", "tail_tiles",
         "tail_inner_iters", "tail_exchange_rounds", "relabel_passes", "orientation", "order", "lambda_chunk",
         "gap", "persist_tiles", "persist_wgs")
SPACE = {
    "tile_w": [32, 64],
    "inner_iters": [4, 8, 12, 16, 32],
    "sweeps_per_relabel": [2, 4, 8, 16],
    "local_bfs_iters": [8, 16, 32, 64],
    "exchange_rounds": [1, 2, 4, 8],
    "tail_tiles": [0, 512, 2048, 8192],
    "tail_inner_iters": [16, 32, 64],
    "tail_exchange_rounds": [4, 16, 32],
    "relabel_passes": [0, 2, 3, 4, 6],
    "orientation": [0, 1, 2, 3],
    "order": [0, 1],
    "lambda_chunk": [0, 1, 2, 4],
    "gap": [0, 1],
    "persist_tiles": [0, 256, 1024, 4096],
    "persist_wgs": [0, 512, 1024],
}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pmf_tune.json")
# the cache committed with the package (written by ``bench.py --tune`` on the device)
PACKAGE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def workload_key(insts: Sequence, device_name: str) -> str:
    """Size class of a batch: log2 buckets of the mean pixel count and of the
    number of solves, the connectivities present and the device."""
    px = sum(i.W * i.H for i in insts) / max(len(insts), 1)
    solves = sum(i.L for i in insts)
    ks = sorted({int(i.K) for i in insts})
    return "px2^%d|solves2^%d|K%s|%s" % (int(math.log2(max(px, 1))), int(math.log2(max(solves, 1))),
                                         "".join(map(str, ks)), device_name)


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0)


def _run(dev_insts, opts: Dict[str, int], repeats: int):
    """(seconds, flows, levels) of one configuration (best of `repeats`)."""
    import torch
    o = pmf.pmf_default_options()
    for k, v in opts.items():
        setattr(o, k, v)
    o.tile_h = 1024 // o.tile_w
    s = pmf.Solver(options=o)
    best = float("inf")
    flows = None
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        flows, status = s.solve(dev_insts)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    levels = []
    for i, d in enumerate(dev_insts):
        out = torch.empty((d.H, d.W), dtype=torch.uint8, device="cuda")
        rc = pmf.pmf_extract_levels(s.handle, i, int(out.data_ptr()))
        if rc != pmf.PMF_OK:
            raise pmf.PmfError(rc, "pmf_extract_levels")
        levels.append(out)
    torch.cuda.synchronize()
    res = (flows.cpu(), [l.cpu() for l in levels], status.cpu())
    s.close()
    return best, res


def _same(a, b) -> bool:
    fa, la, sa = a
    fb, lb, sb = b
    return bool((fa == fb).all()) and all(bool((x == y).all()) for x, y in zip(la, lb)) and bool((sa == sb).all())


def tune(dev_insts: Sequence["pmf.DeviceInstance"], start: Optional[Dict[str, int]] = None, repeats: int = 3,
         space: Optional[Dict[str, List[int]]] = None, log=None, margin: float = 0.03,
         confirm: int = 4) -> Dict[str, object]:
    """Coordinate descent over the knobs on `dev_insts` (device instances).
    A candidate replaces the current point only when it is faster by more
    than `margin` (timings of a solve vary by a few percent from run to run);
    at the end the chosen point and the starting point are timed `confirm`
    more times, interleaved, and the starting point is kept unless the chosen
    one has the lower median.
    Returns {"options": best knob values, "seconds": its time, "trials": [...],
    "rejected": [points whose results differed], "confirmed": {...}}."""
    space = dict(SPACE if space is None else space)
    d = pmf.pmf_default_options()
    cur = {k: int(getattr(d, k)) for k in KNOBS}
    if start:
        cur.update(start)
    t_best, ref = _run(dev_insts, cur, repeats)
    trials = [dict(cur, seconds=t_best)]
    rejected = []
    if log:
        log("tune start %s: %.1f ms" % (cur, t_best * 1e3))
    for knob in KNOBS:
        for v in space.get(knob, []):
            if v == cur[knob]:
                continue
            cand = dict(cur, **{knob: v})
            t, res = _run(dev_insts, cand, repeats)
            ok = _same(res, ref)
            trials.append(dict(cand, seconds=t, same=ok))
            if not ok:
                rejected.append(cand)
                continue
            if log:
                log("tune %s=%s: %.1f ms" % (knob, v, t * 1e3))
            if t < t_best * (1.0 - margin):
                t_best, cur = t, cand
    first = trials[0]
    start_pt = {k: first[k] for k in KNOBS}
    confirmed = None
    if cur != start_pt and confirm > 0:
        ta, tb = [], []
        for _ in range(confirm):
            ta.append(_run(dev_insts, start_pt, 1)[0])
            tb.append(_run(dev_insts, cur, 1)[0])
        ma, mb = sorted(ta)[len(ta) // 2], sorted(tb)[len(tb) // 2]
        confirmed = {"start_ms": round(ma * 1e3, 2), "chosen_ms": round(mb * 1e3, 2)}
        if log:
            log("tune confirm: start %.1f ms, chosen %.1f ms (medians of %d)" % (ma * 1e3, mb * 1e3, confirm))
        if mb >= ma:
            cur, t_best = start_pt, ma
    return {"options": cur, "seconds": t_best, "trials": trials, "rejected": rejected, "confirmed": confirmed}


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, dict], path: str = DEFAULT_CACHE) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def options_for(host_insts: Sequence, dev_insts=None, path: str = DEFAULT_CACHE, retune: bool = False,
                log=None) -> Dict[str, int]:
    """Cached knob values for this workload class; tune (on `dev_insts`) when
    missing or when `retune` is set."""
    key = workload_key(host_insts, _device_name())
    cache = load_cache(path)
    if key in cache and not retune:
        return dict(cache[key]["options"])
    if dev_insts is None:
        return {}
    out = tune(dev_insts, log=log)
    cache[key] = {"options": out["options"], "seconds": out["seconds"], "rejected": out["rejected"]}
    save_cache(cache, path)
    return dict(out["options"])
