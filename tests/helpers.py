"""Shared test helpers: the hand-derived golden fixtures, source-set enumeration
and the checks of a breakpoint list."""

import glob
import json
import os

import numpy as np

from fractions import Fraction

from oracle import oracle as O
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


def source_set_lines(inst):
    """Every source set of a grid of at most 12 pixels as a line in lambda:
    cost(S, lambda) = A_S + w_S * lambda (Sec. 2.1, monotone case), written
    out from the cut definition with Python integers.  Returns the sets
    (bool [2^n, n]) and A, w (object arrays of ints)."""
    Wd, Hd, K = inst.W, inst.H, inst.K
    n = Wd * Hd
    assert n <= 12
    nl = np.asarray(inst.nlink).reshape(K, Hd, Wd)
    cs = np.asarray(inst.cap_src).reshape(-1)
    c0 = np.asarray(inst.cap_snk0).reshape(-1)
    sl = np.asarray(inst.snk_slope).reshape(-1)
    sd = np.asarray(inst.seed).reshape(-1)
    sets = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(bool)
    A, w = [], []
    for T in sets:
        a = b = 0
        for p in range(n):
            if sd[p] == 1:
                a += 0 if T[p] else O.INF
            elif sd[p] == 2:
                a += O.INF if T[p] else 0
            elif T[p]:
                a += int(c0[p])
                b += int(sl[p])
            else:
                a += int(cs[p])
        for k in range(K):
            for y in range(Hd):
                for x in range(Wd):
                    qx, qy = x + O._DX[k], y + O._DY[k]
                    if 0 <= qx < Wd and 0 <= qy < Hd and T[y * Wd + x] and not T[qy * Wd + qx]:
                        a += int(nl[k, y, x])
        A.append(a)
        w.append(b)
    return sets, A, w



def envelope(sets, A, w, lo, hi):
    """Lower envelope over [lo, hi] of the lines A[i] + w[i] * lambda of the
    source sets (minimum cut cost as a function of lambda): its kinks in
    (lo, hi] as Fractions, each piece's line (a, w) and minimal set (the
    intersection of the sets on that line, which the min-cut lattice makes
    optimal)."""
    lines = sorted(set(zip(A, w)))
    def at(l, x):
        return l[0] + l[1] * x
    F = min(at(l, lo) for l in lines)
    cur = min((l for l in lines if at(l, lo) == F), key=lambda l: l[1])
    pieces, bps = [cur], []
    while True:
        cands = [(Fraction(l[0] - cur[0], cur[1] - l[1]), l) for l in lines if l[1] < cur[1]]
        if not cands:
            break
        t = min(c[0] for c in cands)
        if t > hi:
            break
        cur = min((c[1] for c in cands if c[0] == t), key=lambda l: l[1])
        bps.append(t)
        pieces.append(cur)
    A_, w_ = np.array(A, dtype=object), np.array(w, dtype=object)
    psets = []
    for a, b in pieces:
        on = (A_ == a) & (w_ == b)
        psets.append(np.logical_and.reduce(sets[on.astype(bool)], axis=0))
    return bps, pieces, psets


def check_breakpoints_oracle(inst, lo, hi, num, den, pa, pw, ex, threads):
    """A breakpoint list proven exact with the oracle: consecutive pieces meet
    at each breakpoint with strictly falling slopes (a genuine kink), the
    oracle's F equals the pieces' lines at lam_lo, at lam_hi and at every
    breakpoint (F is concave and at most every line, so equal at both ends of
    a piece means equal on all of it: no breakpoint is missed), and the
    oracle's minimal set equals the exit map's set of the piece inside every
    piece and the right-hand piece at every breakpoint."""
    nb = len(num)
    assert len(den) == nb and len(pa) == len(pw) == nb + 1
    xs = [Fraction(int(a), int(b)) for a, b in zip(num, den)]
    for j, x in enumerate(xs):
        assert int(den[j]) >= 1 and np.gcd(int(num[j]), int(den[j])) == 1, j
        assert lo < x <= hi and (j == 0 or xs[j - 1] < x), j
        assert int(pw[j + 1]) < int(pw[j]), j
        assert int(pa[j]) + int(pw[j]) * x == int(pa[j + 1]) + int(pw[j + 1]) * x, j
    ex = np.asarray(ex)
    assert ex.min() >= 0 and ex.max() <= nb + 1
    pts = [(Fraction(lo), 0), (Fraction(hi), nb)]  # (lambda, piece whose minimal set holds there)
    for j, x in enumerate(xs):
        pts.append((x, j + 1))
    ends = [Fraction(lo)] + xs + [Fraction(hi)]
    for j in range(nb + 1):
        if ends[j] < ends[j + 1]:
            pts.append(((ends[j] + ends[j + 1]) / 2, j))
    tasks = [(x.numerator, x.denominator) for x, _ in pts]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as pool:
        sols = list(pool.map(lambda t: O.fifo_pr_rational(inst, t[0], t[1]), tasks))
    for (x, j), (f, m) in zip(pts, sols):
        assert f == (int(pa[j]) + int(pw[j]) * x) * x.denominator, ("F", x, j)
        assert (np.asarray(m).reshape(ex.shape) == (ex > j)).all(), ("set", x, j)
