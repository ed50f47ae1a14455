"""CPU oracle: plain, slow, obviously correct reference for the grid max-flow path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code
with the HIP library and the product never routes through it.

Definitions followed (paper Sec. 2 and 2.1):

* s-t graph: pixels plus source s and sink t; t-links carry the data terms,
  n-links the smoothness terms.  The cost of a cut is the total capacity of
  arcs from the source side to the sink side; a minimum cut has least cost and
  by the Ford-Fulkerson theorem its cost equals the maximum flow value F.
* Monotone parametric case: the sink capacity of a free pixel is
  ``cap_snk0 + slope * lambda`` with ``slope >= 0``; seeds are frozen
  (foreground: source capacity INF, background: sink capacity INF).
* Output per lambda: F and the inclusion-minimal minimum-cut source side S_min
  (the intersection of all minimum cuts; unique).

Functions:

* :func:`fifo_pr`      -- FIFO push-relabel with exact BFS relabelling (C).
* :func:`fifo_pr_rational` -- the same at a rational lambda (capacities scaled by its denominator).
* :func:`ek`           -- Edmonds-Karp shortest augmenting paths (C).
* :func:`cut_cost`     -- cost of a given cut from the original capacities (numpy).
* :func:`brute_force`  -- enumeration of every source set, grids of <= 16 pixels.
* :func:`solve_chain`  -- every lambda of an instance, each solved from scratch.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from typing import List, Sequence, Tuple

import numpy as np

INF = 1 << 30
_DX = (1, -1, 0, 0, 1, -1, -1, 1)
_DY = (0, 0, 1, -1, 1, -1, 1, -1)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with the host C compiler (-O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            for name in ("oracle_fifo_pr", "oracle_ek"):
                fn = getattr(lib, name)
                fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P,
                               ctypes.c_int64, P, P, P]
                fn.restype = ctypes.c_int
            lib.oracle_fifo_pr_rational.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P,
                                                    ctypes.c_int64, ctypes.c_int64, P, P, P]
            lib.oracle_fifo_pr_rational.restype = ctypes.c_int
            lib.oracle_cut_cost.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P,
                                            P, P, ctypes.c_int64, P]
            lib.oracle_cut_cost.restype = ctypes.c_int64
            _lib = lib
    return _lib


def _arrays(inst):
    K, H, W = int(inst.K), int(inst.H), int(inst.W)
    nl = np.ascontiguousarray(inst.nlink, dtype=np.int32).reshape(K, H, W)
    cs = np.ascontiguousarray(inst.cap_src, dtype=np.int32).reshape(H, W)
    c0 = np.ascontiguousarray(inst.cap_snk0, dtype=np.int32).reshape(H, W)
    sl = np.ascontiguousarray(inst.snk_slope, dtype=np.int32).reshape(H, W)
    sd = np.ascontiguousarray(inst.seed, dtype=np.uint8).reshape(H, W)
    return W, H, K, nl, cs, c0, sl, sd


def _call(name: str, inst, lam: int) -> Tuple[int, np.ndarray, np.ndarray]:
    lib = _load()
    W, H, K, nl, cs, c0, sl, sd = _arrays(inst)
    mask = np.zeros((H, W), dtype=np.uint8)
    flow = ctypes.c_int64(0)
    stats = np.zeros(4, dtype=np.int64)
    rc = getattr(lib, name)(W, H, K, nl.ctypes.data, cs.ctypes.data, c0.ctypes.data,
                            sl.ctypes.data, sd.ctypes.data, int(lam), ctypes.addressof(flow),
                            mask.ctypes.data, stats.ctypes.data)
    if rc != 0:
        raise RuntimeError("%s failed with code %d" % (name, rc))
    return int(flow.value), mask.astype(bool), stats


def fifo_pr(inst, lam: int) -> Tuple[int, np.ndarray]:
    """Max-flow value and minimal source side by FIFO push-relabel (int64)."""
    f, m, _ = _call("oracle_fifo_pr", inst, lam)
    return f, m


def fifo_pr_rational(inst, num: int, den: int) -> Tuple[int, np.ndarray]:
    """At lambda = num / den: (den * F(num / den), S_min), by FIFO push-relabel
    on the network with every capacity multiplied by den (INF included), whose
    minimum cuts are the same sets."""
    lib = _load()
    W, H, K, nl, cs, c0, sl, sd = _arrays(inst)
    mask = np.zeros((H, W), dtype=np.uint8)
    flow = ctypes.c_int64(0)
    stats = np.zeros(4, dtype=np.int64)
    rc = lib.oracle_fifo_pr_rational(W, H, K, nl.ctypes.data, cs.ctypes.data, c0.ctypes.data, sl.ctypes.data,
                                     sd.ctypes.data, int(num), int(den), ctypes.addressof(flow), mask.ctypes.data,
                                     stats.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle_fifo_pr_rational failed with code %d" % rc)
    return int(flow.value), mask.astype(bool)


def ek(inst, lam: int) -> Tuple[int, np.ndarray]:
    """Max-flow value and minimal source side by Edmonds-Karp (int64)."""
    f, m, _ = _call("oracle_ek", inst, lam)
    return f, m


def terminal_caps(inst, lam: int) -> Tuple[np.ndarray, np.ndarray]:
    """Source and sink capacities of every pixel at ``lam`` (int64 [H, W])."""
    W, H, K, nl, cs, c0, sl, sd = _arrays(inst)
    src = np.where(sd == 1, INF, np.where(sd == 2, 0, cs)).astype(np.int64)
    snk = np.where(sd == 1, 0, np.where(sd == 2, INF,
                                        c0.astype(np.int64) + sl.astype(np.int64) * int(lam)))
    return src, snk.astype(np.int64)


def cut_cost(inst, lam: int, mask) -> int:
    """c(S) = sum_{p not in S} cs(p) + sum_{p in S} ct(p) + sum_{p in S, q not in S} c(p->q)."""
    W, H, K, nl, cs, c0, sl, sd = _arrays(inst)
    S = np.asarray(mask, dtype=bool).reshape(H, W)
    src, snk = terminal_caps(inst, lam)
    cost = int(src[~S].sum()) + int(snk[S].sum())
    for k in range(K):
        dx, dy = _DX[k], _DY[k]
        y0, y1 = max(0, -dy), H - max(0, dy)
        x0, x1 = max(0, -dx), W - max(0, dx)
        p_in = S[y0:y1, x0:x1]
        q_out = ~S[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
        cost += int(nl[k, y0:y1, x0:x1].astype(np.int64)[p_in & q_out].sum())
    return cost


def cut_cost_c(inst, lam: int, mask) -> int:
    """Same as :func:`cut_cost`, in the C library (for large grids)."""
    lib = _load()
    W, H, K, nl, cs, c0, sl, sd = _arrays(inst)
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(H, W))
    return int(lib.oracle_cut_cost(W, H, K, nl.ctypes.data, cs.ctypes.data, c0.ctypes.data,
                                   sl.ctypes.data, sd.ctypes.data, int(lam), m.ctypes.data))


def brute_force(inst, lam: int):
    """Enumerate all 2^n source sets (n <= 16 pixels).

    Returns ``(F, S_min, argmins)`` where F is the least cut cost, ``argmins``
    is a bool array [count, H, W] of every optimal source set and S_min is
    their intersection.  Raises if the intersection is not itself optimal
    (the minimum cuts of a graph form a lattice, so it must be)."""
    W, H, K, nl, cs, c0, sl, sd = _arrays(inst)
    n = W * H
    if n > 16:
        raise ValueError("brute force limited to 16 pixels")
    src, snk = terminal_caps(inst, lam)
    src = src.reshape(-1)
    snk = snk.reshape(-1)
    codes = np.arange(1 << n, dtype=np.int64)
    T = ((codes[:, None] >> np.arange(n)[None, :]) & 1).astype(bool)  # [2^n, n]
    cost = (np.where(T, 0, src[None, :]) + np.where(T, snk[None, :], 0)).sum(axis=1)
    for k in range(K):
        for y in range(H):
            for x in range(W):
                qx, qy = x + _DX[k], y + _DY[k]
                if not (0 <= qx < W and 0 <= qy < H):
                    continue
                c = int(nl[k, y, x])
                if c == 0:
                    continue
                p, q = y * W + x, qy * W + qx
                cost = cost + c * (T[:, p] & ~T[:, q])
    F = int(cost.min())
    opt = T[cost == F]
    smin = np.logical_and.reduce(opt, axis=0)
    smin_code = int((smin.astype(np.int64) << np.arange(n)).sum())
    if int(cost[smin_code]) != F:
        raise AssertionError("intersection of optimal cuts is not optimal")
    return F, smin.reshape(H, W), opt.reshape(-1, H, W)


def solve_chain(inst, method: str = "fifo_pr") -> Tuple[np.ndarray, np.ndarray]:
    """Every lambda of ``inst`` solved from scratch: (flows int64 [L], masks bool [L, H, W])."""
    fn = fifo_pr if method == "fifo_pr" else ek
    flows, masks = [], []
    for lam in np.asarray(inst.lambdas).tolist():
        f, m = fn(inst, lam)
        flows.append(f)
        masks.append(m)
    return np.array(flows, dtype=np.int64), np.stack(masks)


def solve_many(tasks: Sequence[Tuple[object, int]], threads: int = 0) -> List[Tuple[int, np.ndarray]]:
    """Solve (instance, lambda) tasks on a thread pool, one single-threaded
    solve per task (the trivially parallel scheme of the paper's Sec. 2.2).
    ctypes releases the GIL during each call."""
    threads = threads or (os.cpu_count() or 1)
    _load()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda t: fifo_pr(t[0], t[1]), tasks))
