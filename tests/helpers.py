"""Shared test helpers: the hand-derived golden fixtures."""

import glob
import json
import os

import numpy as np

from paper_1509_06004_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden_instances():
    out = []
    for path in sorted(glob.glob(os.path.join(GOLDEN, "*.json"))):
        with open(path) as f:
            c = json.load(f)
        inst = W.Instance(W=c["W"], H=c["H"], K=c["K"],
                          nlink=np.array(c["nlink"], dtype=np.int32),
                          cap_src=np.array(c["cap_src"], dtype=np.int32),
                          cap_snk0=np.array(c["cap_snk0"], dtype=np.int32),
                          snk_slope=np.array(c["snk_slope"], dtype=np.int32),
                          seed=np.array(c["seed"], dtype=np.uint8),
                          lambdas=np.array(c["lambdas"], dtype=np.int32))
        out.append((c["name"], inst, c["flows"], np.array(c["masks"], dtype=bool)))
    return out


def host_threads() -> int:
    """Worker threads for oracle pools: the CPUs this process may run on,
    at most 16 (one GPU's share of a multi-GPU host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def headroom_instance(rng, Wd, Hd, K, L):
    """Every on-grid n-link at PMF_NLINK_MAX(K), foreground seeds (source
    capacity INF) scattered among free pixels whose source capacities reach
    INF, background seeds on the border ring: excess can reach
    INF + K * PMF_NLINK_MAX(K), just below 2^31."""
    nlmax = ((1 << 30) - 1) // K
    inst = W.tiny_random(rng, Wd, Hd, K, cmax=10, L=L, p_seed=0.2)
    on = inst.nlink != 0
    for k in range(K):
        dx, dy = W.DX[k], W.DY[k]
        ys, xs = np.mgrid[0:Hd, 0:Wd]
        on[k] = (xs + dx >= 0) & (xs + dx < Wd) & (ys + dy >= 0) & (ys + dy < Hd)
    inst.nlink = np.where(on, nlmax, 0).astype(np.int32)
    inst.cap_src = np.where(rng.random((Hd, Wd)) < 0.3, 1 << 30, inst.cap_src).astype(np.int32)
    inst.cap_snk0 = np.where(rng.random((Hd, Wd)) < 0.3, (1 << 30) - 4096, inst.cap_snk0).astype(np.int32)
    inst.snk_slope = rng.integers(0, 3, size=(Hd, Wd)).astype(np.int32)
    inst.lambdas = np.sort(rng.integers(0, 1000, size=L)).astype(np.int32)
    seed = inst.seed.copy()
    seed[0, :] = seed[-1, :] = 2
    seed[:, 0] = seed[:, -1] = 2
    inst.seed = seed
    return inst
