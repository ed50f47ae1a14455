"""Seeded synthetic segmentation workloads (inputs only).

This module draws the grid graphs that both the HIP path and the CPU oracle
consume.  It holds none of the method's arithmetic: it only produces the
capacities of the problem statement (Sec. 2: pixel vertices, terminal links as
data terms, neighbour links as smoothness terms; Sec. 2.1: frozen seeds and a
log-spaced lambda schedule) as int32/uint8 host arrays.

Conventions shared with the C ABI (``include/pmf.h``):

* Direction ``k`` has offset ``(DX[k], DY[k])``; ``k ^ 1`` is the opposite one.
  4-connectivity uses directions 0..3, 8-connectivity 0..7.
* ``nlink[k, y, x]`` is the capacity of the arc from pixel ``(x, y)`` to pixel
  ``(x + DX[k], y + DY[k])``; it is 0 where that neighbour is off the grid.
* ``seed[y, x]``: 0 free pixel, 1 foreground seed (tied to the source with
  ``INF``), 2 background seed (tied to the sink with ``INF``).
* A free pixel has source capacity ``cap_src`` and sink capacity
  ``cap_snk0 + snk_slope * lambda`` (the monotone parametric case of Sec. 2.1).
* ``INF = 2**30``.

The stand-in for the paper's VOC2012 images (which are not available here) is
a Voronoi mosaic with uniform grey levels plus Gaussian noise; sizes, seed
layouts and lambda schedules follow the paper's workloads (Sec. 3.3.2: half
downsampled VOC images; Sec. 4.1: 20 lambda values per seed).
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

INF = 1 << 30
MASTER_SEED = 1509060040

DX = (1, -1, 0, 0, 1, -1, -1, 1)
DY = (0, 0, 1, -1, 1, -1, 1, -1)


@dataclasses.dataclass
class Instance:
    """One (image, seed) problem with its lambda schedule (host arrays)."""

    W: int
    H: int
    K: int
    nlink: np.ndarray      # int32 [K, H, W]
    cap_src: np.ndarray    # int32 [H, W]
    cap_snk0: np.ndarray   # int32 [H, W]
    snk_slope: np.ndarray  # int32 [H, W]
    seed: np.ndarray       # uint8 [H, W]
    lambdas: np.ndarray    # int32 [L], non-decreasing
    image: int = 0         # images sharing ``image`` share ``nlink``

    @property
    def L(self) -> int:
        return int(self.lambdas.shape[0])

    @property
    def n(self) -> int:
        return self.W * self.H

    def with_lambdas(self, lambdas) -> "Instance":
        return dataclasses.replace(self, lambdas=np.ascontiguousarray(lambdas, dtype=np.int32))


def rng_for(cfg: int, idx: int) -> np.random.Generator:
    return np.random.default_rng([MASTER_SEED, cfg, idx])


def round_half_away(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def voronoi_image(W: int, H: int, R: int, rng: np.random.Generator,
                  noise: float = 0.02) -> np.ndarray:
    """Grey image in [0,1]: nearest of R uniform sites, uniform grey per region,
    N(0, noise^2) per pixel, clipped.  Ties go to the lowest site index."""
    sites = rng.uniform(0.0, 1.0, size=(R, 2)) * np.array([W, H], dtype=np.float64)
    grey = rng.uniform(0.0, 1.0, size=R)
    xs = np.arange(W, dtype=np.float64) + 0.5
    ys = np.arange(H, dtype=np.float64) + 0.5
    best = np.full((H, W), np.inf)
    lab = np.zeros((H, W), dtype=np.int64)
    for r in range(R):
        d2 = (xs[None, :] - sites[r, 0]) ** 2 + (ys[:, None] - sites[r, 1]) ** 2
        upd = d2 < best  # strict: an equal later site does not win
        best = np.where(upd, d2, best)
        lab = np.where(upd, r, lab)
    img = grey[lab] + rng.normal(0.0, noise, size=(H, W))
    return np.clip(img, 0.0, 1.0)


def nlinks(img: np.ndarray, K: int, scale: float = 1000.0, sigma2: float = 0.01) -> np.ndarray:
    """Smoothness capacities rint(scale * exp(-(I_p - I_q)^2 / sigma2)); the
    diagonal ones of 8-connectivity are divided by sqrt(2) before rounding.
    Symmetric; zero towards off-grid neighbours."""
    H, W = img.shape
    out = np.zeros((K, H, W), dtype=np.int32)
    for k in range(K):
        dx, dy = DX[k], DY[k]
        y0, y1 = max(0, -dy), H - max(0, dy)
        x0, x1 = max(0, -dx), W - max(0, dx)
        p = img[y0:y1, x0:x1]
        q = img[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
        w = scale * np.exp(-((p - q) ** 2) / sigma2)
        if dx != 0 and dy != 0:
            w = w / math.sqrt(2.0)
        out[k, y0:y1, x0:x1] = np.rint(w).astype(np.int32)
    return out


def border_mask(W: int, H: int) -> np.ndarray:
    m = np.zeros((H, W), dtype=bool)
    m[0, :] = m[-1, :] = True
    m[:, 0] = m[:, -1] = True
    return m


_CONST = {}


def const_plane(H: int, W: int, value: int) -> np.ndarray:
    """Read-only int32 plane shared by every instance of that shape."""
    key = (H, W, value)
    if key not in _CONST:
        a = np.full((H, W), value, dtype=np.int32)
        a.flags.writeable = False
        _CONST[key] = a
    return _CONST[key]


def seed_instance(img: np.ndarray, nl: np.ndarray, K: int, cx: int, cy: int, side: int,
                  lambdas: Sequence[int], image: int = 0, src_scale: float = 200.0) -> Instance:
    """Foreground seed = side x side square centred at (cx, cy); background seed
    = the border ring.  Free pixels: cap_src = rint(src_scale*(1-|I - mean I over seed|)),
    cap_snk0 = 0, slope 1 (sink capacity = lambda)."""
    H, W = img.shape
    half = side // 2
    seed = np.zeros((H, W), dtype=np.uint8)
    ys = slice(max(0, cy - half), min(H, cy - half + side))
    xs = slice(max(0, cx - half), min(W, cx - half + side))
    seed[ys, xs] = 1
    bm = border_mask(W, H)
    seed[bm] = 2  # the generator keeps seeds off the border ring anyway
    iseed = float(img[ys, xs].mean())
    cap_src = np.rint(src_scale * (1.0 - np.abs(img - iseed))).astype(np.int32)
    free = seed == 0
    cap_src = np.where(free, cap_src, 0).astype(np.int32)
    # sink capacity lambda for free pixels; seeds ignore these two planes, so
    # every instance of the image shares them
    return Instance(W=W, H=H, K=K, nlink=nl, cap_src=cap_src, cap_snk0=const_plane(H, W, 0),
                    snk_slope=const_plane(H, W, 1), seed=seed,
                    lambdas=np.ascontiguousarray(lambdas, dtype=np.int32), image=image)


def geometric_lambdas(lo: float, hi: float, L: int) -> np.ndarray:
    """lambda_k = lo * (hi/lo)^(k/(L-1)) in float64, rounded half away from zero.
    Duplicates are kept (the schedule 1..2000 with L=20 starts 1, 1, 2, 3, ...)."""
    if L == 1:
        return np.array([int(round_half_away(lo))], dtype=np.int32)
    k = np.arange(L, dtype=np.float64)
    lam = lo * (hi / lo) ** (k / (L - 1))
    return round_half_away(lam).astype(np.int32)


def loguniform_lambdas(rng: np.random.Generator, L: int, hi: float = 5000.0) -> np.ndarray:
    lam = np.exp(rng.uniform(0.0, math.log(hi), size=L))
    return np.sort(np.rint(lam)).astype(np.int32)


# ---------------------------------------------------------------------------
# The five workloads.
# ---------------------------------------------------------------------------

def config0() -> List[Instance]:
    """64x64, 4-connected, 8 regions, 5x5 centre seed, one lambda = 100."""
    rng = rng_for(0, 0)
    img = voronoi_image(64, 64, 8, rng)
    nl = nlinks(img, 4)
    return [seed_instance(img, nl, 4, 32, 32, 5, [100])]


def config1() -> List[Instance]:
    """320x240, 4-connected, 16 regions, 5x5 centre seed, 20 geometric lambdas 1..2000."""
    rng = rng_for(1, 0)
    W, H = 320, 240
    img = voronoi_image(W, H, 16, rng)
    nl = nlinks(img, 4)
    return [seed_instance(img, nl, 4, W // 2, H // 2, 5, geometric_lambdas(1, 2000, 20))]


def lattice_centres(W: int, H: int, m: int = 5) -> List[tuple]:
    out = []
    for j in range(m):
        for i in range(m):
            cx = int(math.floor((i + 1) * W / (m + 1) + 0.5))
            cy = int(math.floor((j + 1) * H / (m + 1) + 0.5))
            out.append((cx, cy))
    return out


def config2(K: int = 8, seeds: Optional[int] = None, L: int = 20) -> List[Instance]:
    """500x375, K-connected (8 as specified; 4 for the headline metric), 24 regions,
    25 seeds (7x7 squares on a 5x5 lattice) x 20 geometric lambdas 1..2000."""
    rng = rng_for(2, 0)
    W, H = 500, 375
    img = voronoi_image(W, H, 24, rng)
    nl = nlinks(img, K)
    lam = geometric_lambdas(1, 2000, L)
    insts = [seed_instance(img, nl, K, cx, cy, 7, lam) for cx, cy in lattice_centres(W, H)]
    return insts if seeds is None else insts[:seeds]


def random_image_instances(rng: np.random.Generator, image: int, wmin: int, wmax: int,
                           hmin: int, hmax: int, smax: int, cfg_scale: float = 1.0) -> List[Instance]:
    W = int(rng.integers(wmin, wmax + 1))
    H = int(rng.integers(hmin, hmax + 1))
    K = 4 if rng.integers(0, 2) == 0 else 8
    R = int(rng.integers(8, 49))
    img = voronoi_image(W, H, R, rng)
    nl = nlinks(img, K)
    S = int(rng.integers(1, smax + 1))
    out = []
    for _ in range(S):
        cx = int(rng.integers(4, W - 4))
        cy = int(rng.integers(4, H - 4))
        L = int(rng.integers(10, 31))
        out.append(seed_instance(img, nl, K, cx, cy, 7, loguniform_lambdas(rng, L), image=image))
    return out


def config3(images: int = 256, wmax: int = 640, hmax: int = 480) -> List[Instance]:
    """Uneven sizes: per image W~U{64..640}, H~U{64..480}, K by coin flip,
    8..48 regions, 1..16 seeds (7x7, off the border ring), 10..30 log-uniform
    lambdas in [1, 5000]."""
    out = []
    for i in range(images):
        rng = rng_for(3, i)
        out.extend(random_image_instances(rng, i, 64, wmax, 64, hmax, 16))
    return out


def config4_stream(qps: float, seconds: float, warmup_s: float = 0.0, templates: int = 24):
    """Serving workload: Poisson arrivals at `qps` over warmup_s + seconds; each
    request is one image (W in 128..640, H in 96..480, K by coin flip, 8..48
    regions) with 1..32 seeds, each with its own 10..30-point schedule in
    [1, 5000].  Requests are drawn from a pool of `templates` generated images
    (drawing a fresh 640x480 image per request would take longer than serving
    it); arrival times and template choice are seeded by the QPS.

    Returns (arrival times [n], template index [n], template list)."""
    rng = np.random.default_rng([MASTER_SEED, 4, int(round(qps))])
    t, arr = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / qps))
        if t >= warmup_s + seconds:
            break
        arr.append(t)
    pick = rng.integers(0, templates, size=len(arr))
    pool = [random_image_instances(rng_for(4, 1000 + i), i, 128, 640, 96, 480, 32) for i in range(templates)]
    return np.array(arr, dtype=np.float64), pick, pool


def tiny_random(rng: np.random.Generator, W: int, H: int, K: int, cmax: int = 20,
                L: int = 1, p_seed: float = 0.15, p_inf_nlink: float = 0.0,
                lam_max: int = 30) -> Instance:
    """Small random grid with arbitrary (asymmetric) capacities in 0..cmax,
    random fg/bg seeds and a random non-decreasing schedule.  Used to pin the
    oracle by brute force and to cover odd shapes in parity tests."""
    nl = rng.integers(0, cmax + 1, size=(K, H, W)).astype(np.int32)
    if p_inf_nlink > 0:
        big = rng.random((K, H, W)) < p_inf_nlink
        nl = np.where(big, 1 << 20, nl).astype(np.int32)
    for k in range(K):
        dx, dy = DX[k], DY[k]
        if dx > 0:
            nl[k, :, W - dx:] = 0
        if dx < 0:
            nl[k, :, :-dx] = 0
        if dy > 0:
            nl[k, H - dy:, :] = 0
        if dy < 0:
            nl[k, :-dy, :] = 0
    u = rng.random((H, W))
    seed = np.zeros((H, W), dtype=np.uint8)
    seed[u < p_seed] = 1
    seed[(u >= p_seed) & (u < 2 * p_seed)] = 2
    cap_src = rng.integers(0, cmax + 1, size=(H, W)).astype(np.int32)
    cap_snk0 = rng.integers(0, cmax + 1, size=(H, W)).astype(np.int32)
    slope = rng.integers(0, 3, size=(H, W)).astype(np.int32)
    lam = np.sort(rng.integers(0, lam_max + 1, size=L)).astype(np.int32)
    return Instance(W=W, H=H, K=K, nlink=nl, cap_src=cap_src, cap_snk0=cap_snk0,
                    snk_slope=slope, seed=seed, lambdas=lam)
