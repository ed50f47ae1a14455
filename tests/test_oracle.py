"""Pins of the CPU oracle against what the problem statement and mathematics fix.

The paper prints no worked example, so the oracle is pinned by
* hand-derived cuts (``tests/golden``), checked against the definition of the
  cut cost (Sec. 2),
* exhaustive enumeration of every source set on grids of at most 16 pixels,
* two independent algorithms (push-relabel on an arc list, Edmonds-Karp on
  residual planes),
* the duality certificate F == cost(S_min) (max flow = min cut, Sec. 2),
* closed forms (no smoothness arcs; unbreakable smoothness arcs; one pixel),
* nesting and concavity across an increasing lambda (monotone case, Sec. 2.1),
* metamorphic relations (scaling, a constant on both terminal arcs, the s-t
  swap of Sec. 3.2, the supergraph union of Sec. 3.1).
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_06004_amd import workload as W

from helpers import golden_instances, source_set_lines


@pytest.mark.parametrize("name,inst,flows,masks", golden_instances(),
                         ids=[g[0] for g in golden_instances()])
def test_golden_hand_derived(name, inst, flows, masks):
    for k, lam in enumerate(inst.lambdas.tolist()):
        assert O.cut_cost(inst, lam, masks[k]) == flows[k]
        F, S, _ = O.brute_force(inst, lam)
        assert F == flows[k] and (S == masks[k]).all()
        for fn in (O.fifo_pr, O.ek):
            f, m = fn(inst, lam)
            assert f == flows[k], (fn.__name__, lam)
            assert (m == masks[k]).all(), (fn.__name__, lam)


def _random_tiny(seed, count):
    rng = np.random.default_rng(seed)
    for i in range(count):
        Wd = int(rng.integers(1, 5))
        Hd = int(rng.integers(1, 5))
        K = 4 if i % 2 == 0 else 8
        cmax = int(rng.choice([1, 2, 3, 8, 24]))  # small capacities make ties frequent
        yield W.tiny_random(rng, Wd, Hd, K, cmax=cmax, L=3, lam_max=3 * cmax,
                            p_seed=float(rng.uniform(0, 0.3)),
                            p_inf_nlink=0.1 if i % 5 == 0 else 0.0)


def test_brute_force_vs_both_algorithms():
    """Every grid of at most 4x4: F and S_min exactly equal to the enumeration."""
    checked = 0
    for inst in _random_tiny(11, 400):
        for lam in inst.lambdas.tolist():
            F, S, opt = O.brute_force(inst, lam)
            f1, m1 = O.fifo_pr(inst, lam)
            f2, m2 = O.ek(inst, lam)
            assert f1 == F and f2 == F
            assert (m1 == S).all() and (m2 == S).all()
            checked += 1
    assert checked == 1200


def test_brute_force_ties_are_common():
    """The random tiny cases must exercise several optimal cuts (so S_min is a
    real choice, not the only optimum)."""
    multi = 0
    for inst in _random_tiny(12, 200):
        lam = int(inst.lambdas[0])
        _, _, opt = O.brute_force(inst, lam)
        multi += opt.shape[0] > 1
    assert multi >= 25


def test_single_pixel():
    for cs, ct in [(0, 0), (5, 3), (3, 5), (7, 7)]:
        inst = W.Instance(W=1, H=1, K=4, nlink=np.zeros((4, 1, 1), np.int32),
                          cap_src=np.array([[cs]], np.int32), cap_snk0=np.array([[ct]], np.int32),
                          snk_slope=np.zeros((1, 1), np.int32), seed=np.zeros((1, 1), np.uint8),
                          lambdas=np.array([0], np.int32))
        for fn in (O.fifo_pr, O.ek):
            f, m = fn(inst, 0)
            assert f == min(cs, ct)
            assert bool(m[0, 0]) == (cs > ct)  # ties go to the sink side


def _zero_offgrid(nl, Wd, Hd):
    for k in range(nl.shape[0]):
        dx, dy = W.DX[k], W.DY[k]
        if dx > 0:
            nl[k, :, Wd - dx:] = 0
        if dx < 0:
            nl[k, :, :-dx] = 0
        if dy > 0:
            nl[k, Hd - dy:, :] = 0
        if dy < 0:
            nl[k, :-dy, :] = 0


@pytest.mark.parametrize("K", [4, 8])
def test_closed_form_no_smoothness(K):
    """Zero n-links: F = sum min(cs, ct), S_min = {cs > ct}."""
    rng = np.random.default_rng(21 + K)
    inst = W.tiny_random(rng, 37, 23, K, cmax=50, L=4, p_seed=0.05)
    inst.nlink[:] = 0
    for lam in inst.lambdas.tolist():
        cs, ct = O.terminal_caps(inst, lam)
        for fn in (O.fifo_pr, O.ek):
            f, m = fn(inst, lam)
            assert f == int(np.minimum(cs, ct).sum())
            assert (m == (cs > ct)).all()


@pytest.mark.parametrize("K", [4, 8])
def test_closed_form_unbreakable_smoothness(K):
    """Every n-link larger than the sum of all t-links (no seeds): the grid moves
    as one block, F = min(sum cs, sum ct), S_min = all if sum cs > sum ct else none."""
    rng = np.random.default_rng(31 + K)
    for trial in range(6):
        inst = W.tiny_random(rng, 9, 7, K, cmax=30, L=1, p_seed=0.0)
        inst.snk_slope[:] = 0
        if trial == 5:  # an exact tie goes to the sink side
            inst.cap_snk0[:] = inst.cap_src
        cs, ct = O.terminal_caps(inst, 0)
        inst.nlink[:] = int(cs.sum() + ct.sum()) + 1
        _zero_offgrid(inst.nlink, 9, 7)
        for fn in (O.fifo_pr, O.ek):
            f, m = fn(inst, 0)
            assert f == min(int(cs.sum()), int(ct.sum()))
            assert (m == (cs.sum() > ct.sum())).all()


def test_fifo_pr_vs_ek_midsize():
    """Two independent algorithms agree on F and S_min on grids up to 64x64."""
    rng = np.random.default_rng(41)
    for i in range(6):
        K = 4 if i % 2 == 0 else 8
        inst = W.tiny_random(rng, int(rng.integers(20, 65)), int(rng.integers(20, 65)), K,
                             cmax=int(rng.integers(5, 200)), L=2, p_seed=0.02)
        for lam in inst.lambdas.tolist():
            f1, m1 = O.fifo_pr(inst, lam)
            f2, m2 = O.ek(inst, lam)
            assert f1 == f2 and (m1 == m2).all()
    c0 = W.config0()[0]
    f1, m1 = O.fifo_pr(c0, 100)
    f2, m2 = O.ek(c0, 100)
    assert f1 == f2 and (m1 == m2).all()
    assert O.cut_cost(c0, 100, m1) == f1


def check_chain(inst, flows, masks):
    """Duality, nesting, the derivative sandwich and concavity for one schedule."""
    lams = inst.lambdas.astype(np.int64)
    slope = np.where(inst.seed == 0, inst.snk_slope, 0).astype(np.int64)
    for k in range(len(lams)):
        # duality certificate: a flow value equal to a cut cost proves both optimal
        assert O.cut_cost_c(inst, int(lams[k]), masks[k]) == flows[k]
        if k == 0:
            continue
        d = int(lams[k] - lams[k - 1])
        # nesting of optimal source sets (monotone case)
        assert not (masks[k] & ~masks[k - 1]).any()
        # F grows, by at most w(S_{k-1}) * d and at least w(S_k) * d
        df = int(flows[k] - flows[k - 1])
        assert int(slope[masks[k]].sum()) * d <= df <= int(slope[masks[k - 1]].sum()) * d
    # concavity in lambda on distinct points
    pts = [(int(l), int(f)) for l, f in zip(lams, flows)]
    for (l0, f0), (l1, f1), (l2, f2) in zip(pts, pts[1:], pts[2:]):
        if l0 < l1 < l2:
            assert (f1 - f0) * (l2 - l1) >= (f2 - f1) * (l1 - l0)


def test_chain_invariants_config1():
    inst = W.config1()[0]
    flows, masks = O.solve_chain(inst)
    check_chain(inst, flows, masks)
    assert masks[0].sum() > masks[-1].sum()  # the schedule does move the cut


def test_chain_invariants_random_midsize():
    rng = np.random.default_rng(51)
    for i in range(4):
        inst = W.tiny_random(rng, 40, 30, 4 if i % 2 else 8, cmax=60, L=8, p_seed=0.03, lam_max=80)
        flows, masks = O.solve_chain(inst)
        check_chain(inst, flows, masks)


def test_metamorphic_scale_and_shift():
    rng = np.random.default_rng(61)
    for i in range(10):
        K = 4 if i % 2 else 8
        inst = W.tiny_random(rng, 12, 9, K, cmax=40, L=1, p_seed=0.0)
        lam = int(inst.lambdas[0])
        f, m = O.fifo_pr(inst, lam)
        k = 3
        sc = W.Instance(W=inst.W, H=inst.H, K=K, nlink=inst.nlink * k, cap_src=inst.cap_src * k,
                        cap_snk0=inst.cap_snk0 * k, snk_slope=inst.snk_slope * k, seed=inst.seed,
                        lambdas=inst.lambdas)
        f2, m2 = O.fifo_pr(sc, lam)
        assert f2 == k * f and (m2 == m).all()
        # add c to both terminal arcs of one free pixel: F + c, same S_min
        y, x = int(rng.integers(0, 9)), int(rng.integers(0, 12))
        sh = W.Instance(W=inst.W, H=inst.H, K=K, nlink=inst.nlink, cap_src=inst.cap_src.copy(),
                        cap_snk0=inst.cap_snk0.copy(), snk_slope=inst.snk_slope, seed=inst.seed,
                        lambdas=inst.lambdas)
        sh.cap_src[y, x] += 17
        sh.cap_snk0[y, x] += 17
        f3, m3 = O.fifo_pr(sh, lam)
        assert f3 == f + 17 and (m3 == m).all()


def swap_instance(inst, lam):
    """Reverse every arc and exchange s and t (the s-t swap of Sec. 3.2), at a
    fixed lambda: the sink capacity becomes a lambda-free source capacity."""
    K, H, Wd = inst.K, inst.H, inst.W
    cs, ct = O.terminal_caps(inst, lam)
    nl = np.zeros_like(inst.nlink)
    for k in range(K):
        dx, dy = W.DX[k], W.DY[k]
        y0, y1 = max(0, -dy), H - max(0, dy)
        x0, x1 = max(0, -dx), Wd - max(0, dx)
        # reversed arc p -> q carries the capacity of q -> p (direction k^1 at q)
        nl[k, y0:y1, x0:x1] = inst.nlink[k ^ 1, y0 + dy:y1 + dy, x0 + dx:x1 + dx]
    seed = np.where(inst.seed == 1, 2, np.where(inst.seed == 2, 1, 0)).astype(np.uint8)
    return W.Instance(W=Wd, H=H, K=K, nlink=nl,
                      cap_src=np.where(inst.seed == 0, ct, 0).astype(np.int32),
                      cap_snk0=np.where(inst.seed == 0, cs, 0).astype(np.int32),
                      snk_slope=np.zeros_like(inst.snk_slope), seed=seed,
                      lambdas=np.array([0], np.int32))


def test_metamorphic_st_swap():
    """The s-t swap keeps the flow value; the swapped graph's minimal source side
    is the complement of the original's maximal source side (on tiny grids the
    maximal side is the union of all optima found by enumeration)."""
    for inst in _random_tiny(72, 120):
        lam = int(inst.lambdas[1])
        f, m = O.fifo_pr(inst, lam)
        sw = swap_instance(inst, lam)
        f2, m2 = O.fifo_pr(sw, 0)
        assert f2 == f
        _, _, opt = O.brute_force(inst, lam)
        smax = np.logical_or.reduce(opt, axis=0)
        assert (~m2 == smax).all()
    big = W.config0()[0]
    f, m = O.fifo_pr(big, 100)
    sw = swap_instance(big, 100)
    f2, m2 = O.fifo_pr(sw, 0)
    assert f2 == f and O.cut_cost(big, 100, ~m2) == f and not (m & m2).any()


def test_supergraph_union():
    """Two graphs knitted side by side through a column of isolated vertices with
    zero-capacity arcs (Sec. 3.1): the union's F is the sum and its S_min is the
    union of the parts' S_min."""
    rng = np.random.default_rng(81)
    for K in (4, 8):
        a = W.tiny_random(rng, 11, 8, K, cmax=30, L=1, p_seed=0.1)
        b = W.tiny_random(rng, 7, 8, K, cmax=30, L=1, p_seed=0.1)
        b.lambdas[:] = a.lambdas
        lam = int(a.lambdas[0])
        Wd = a.W + 1 + b.W

        def cat(x, y, fill):
            mid = np.full(x.shape[:-1] + (1,), fill, dtype=x.dtype)
            return np.concatenate([x, mid, y], axis=-1)

        u = W.Instance(W=Wd, H=8, K=K, nlink=cat(a.nlink, b.nlink, 0),
                       cap_src=cat(a.cap_src, b.cap_src, 0),
                       cap_snk0=cat(a.cap_snk0, b.cap_snk0, 0),
                       snk_slope=cat(a.snk_slope, b.snk_slope, 0),
                       seed=cat(a.seed, b.seed, 0), lambdas=a.lambdas)
        fa, ma = O.fifo_pr(a, lam)
        fb, mb = O.fifo_pr(b, lam)
        fu, mu = O.fifo_pr(u, lam)
        assert fu == fa + fb
        assert (mu[:, :a.W] == ma).all() and (mu[:, a.W + 1:] == mb).all()
        assert not mu[:, a.W].any()


def test_cut_cost_c_matches_numpy():
    rng = np.random.default_rng(91)
    for K in (4, 8):
        inst = W.tiny_random(rng, 30, 20, K, cmax=100, L=1)
        m = rng.random((20, 30)) < 0.5
        assert O.cut_cost_c(inst, 7, m) == O.cut_cost(inst, 7, m)


def test_planted_mistake_is_caught():
    """A plausible slip in the cut-cost definition (counting arcs entering the
    source side instead of leaving it) fails the hand-derived fixtures."""
    def wrong_cost(inst, lam, mask):
        S = np.asarray(mask, bool)
        cs, ct = O.terminal_caps(inst, lam)
        cost = int(cs[~S].sum()) + int(ct[S].sum())
        H, Wd = S.shape
        for k in range(inst.K):
            for y in range(H):
                for x in range(Wd):
                    qx, qy = x + W.DX[k], y + W.DY[k]
                    if 0 <= qx < Wd and 0 <= qy < H and (not S[y, x]) and S[qy, qx]:
                        cost += int(inst.nlink[k, y, x])
        return cost
    bad = 0
    for name, inst, flows, masks in golden_instances():
        for k, lam in enumerate(inst.lambdas.tolist()):
            bad += wrong_cost(inst, lam, masks[k]) != flows[k]
    assert bad > 0


def test_int32_headroom_brute_force():
    """At the largest admitted n-link capacity next to INF seeds (excess up to
    INF + K * PMF_NLINK_MAX(K)), both algorithms equal exhaustive enumeration:
    the oracle's int64 arithmetic holds where the device's int32 state is
    tightest."""
    from helpers import headroom_instance
    rng = np.random.default_rng(2024)
    biggest = 0
    for i in range(24):
        K = 4 if i % 2 else 8
        Wd, Hd = int(rng.integers(3, 5)), int(rng.integers(3, 5))
        inst = headroom_instance(rng, Wd, Hd, K, 2)
        for lam in inst.lambdas.tolist():
            F, S, _ = O.brute_force(inst, lam)
            biggest = max(biggest, F)
            for fn in (O.fifo_pr, O.ek):
                f, m = fn(inst, lam)
                assert f == F and (m == S).all(), (i, fn.__name__, lam)
    assert biggest >= (1 << 31) - 8  # some optimal cuts cost about INF + K * PMF_NLINK_MAX(K)


def test_rational_lambda_brute_force():
    """At rational lambda = num/den the scaled solve gives den * F and S_min
    exactly as the enumeration of every source set in exact rational
    arithmetic; den = 1 is the integer solve."""
    from fractions import Fraction
    rng = np.random.default_rng(515)
    checked = 0
    for i, inst in enumerate(_random_tiny(33, 60)):
        if inst.W * inst.H > 12:
            continue
        sets, A, w = source_set_lines(inst)
        for _ in range(4):
            den = int(rng.integers(1, 8))
            num = int(rng.integers(0, 30 * den))
            lam = Fraction(num, den)
            cost = [a + b * lam for a, b in zip(A, w)]
            F = min(cost)
            smin = np.logical_and.reduce(sets[[c == F for c in cost]], axis=0)
            f, m = O.fifo_pr_rational(inst, num, den)
            assert f == F * den, (i, num, den)
            assert (m.reshape(-1) == smin).all(), (i, num, den)
            if den == 1:
                f1, m1 = O.fifo_pr(inst, num)
                assert f1 == f and (m1 == m).all()
            checked += 1
    assert checked >= 150
    # capacities near INF (n-links at PMF_NLINK_MAX next to INF seeds): a
    # cut through an INF arc competes with finite ones only if INF is scaled
    # with everything else
    from helpers import headroom_instance
    big = 0
    for i in range(12):
        inst = headroom_instance(rng, 3, int(rng.integers(3, 5)), 4 if i % 2 else 8, 1)
        sets, A, w = source_set_lines(inst)
        for den in (2, 3, 5):
            num = int(rng.integers(0, 1000 * den))
            lam = Fraction(num, den)
            cost = [a + b * lam for a, b in zip(A, w)]
            F = min(cost)
            smin = np.logical_and.reduce(sets[[c == F for c in cost]], axis=0)
            f, m = O.fifo_pr_rational(inst, num, den)
            assert f == F * den and (m.reshape(-1) == smin).all(), (i, num, den)
            big = max(big, f)
    assert big > (1 << 31)  # scaled cuts well above INF: INF must scale with them


def test_envelope_of_enumeration_passes_the_oracle_check():
    """The two checks of a breakpoint list agree: the lower envelope of every
    source set's line, turned into breakpoints, pieces and exit pieces, passes
    the oracle-based proof at rational lambdas."""
    from helpers import check_breakpoints_oracle, envelope
    rng = np.random.default_rng(616)
    total = 0
    for i in range(60):
        Wd, Hd = int(rng.integers(1, 4)), int(rng.integers(1, 5))
        inst = W.tiny_random(rng, Wd, Hd, 4 if i % 2 else 8, cmax=int(rng.choice([5, 20, 60])), L=1,
                             p_seed=float(rng.uniform(0, 0.2)))
        lo, hi = int(rng.integers(0, 4)), int(rng.integers(20, 120))
        sets, A, w = source_set_lines(inst)
        bps, pieces, psets = envelope(sets, A, w, lo, hi)
        ex = np.full(Wd * Hd, len(bps) + 1, dtype=np.int64)
        for j in range(len(psets) - 1, -1, -1):
            ex[~psets[j]] = j
        num = np.array([b.numerator for b in bps], dtype=np.int64)
        den = np.array([b.denominator for b in bps], dtype=np.int64)
        pa = np.array([a for a, _ in pieces], dtype=np.int64)
        pw = np.array([b for _, b in pieces], dtype=np.int64)
        check_breakpoints_oracle(inst, lo, hi, num, den, pa, pw, ex.reshape(Hd, Wd), 4)
        total += len(bps)
    assert total >= 25


def test_breakpoint_check_rejects_planted_mistakes():
    """The oracle-based proof of a breakpoint list fails on a list with a
    breakpoint dropped, a breakpoint moved, a piece's slope changed, or a
    pixel's exit piece changed."""
    from helpers import check_breakpoints_oracle, envelope
    rng = np.random.default_rng(31)
    for _ in range(200):
        Wd, Hd = int(rng.integers(2, 4)), int(rng.integers(2, 4))
        inst = W.tiny_random(rng, Wd, Hd, 4, cmax=60, L=1, p_seed=0.0)
        sets, A, w = source_set_lines(inst)
        bps, pieces, psets = envelope(sets, A, w, 0, 100)
        if len(bps) >= 2:
            break
    assert len(bps) >= 2
    ex = np.full(Wd * Hd, len(bps) + 1, dtype=np.int64)
    for j in range(len(psets) - 1, -1, -1):
        ex[~psets[j]] = j
    num = [b.numerator for b in bps]
    den = [b.denominator for b in bps]
    pa = [a for a, _ in pieces]
    pw = [b for _, b in pieces]
    good = (num, den, pa, pw, ex)

    def check(num, den, pa, pw, ex):
        check_breakpoints_oracle(inst, 0, 100, np.array(num, dtype=np.int64), np.array(den, dtype=np.int64),
                                 np.array(pa, dtype=np.int64), np.array(pw, dtype=np.int64),
                                 np.asarray(ex).reshape(Hd, Wd), 2)

    check(*good)
    bad = [
        (num[1:], den[1:], pa[1:], pw[1:], np.maximum(ex - 1, 0)),   # first breakpoint dropped
        ([num[0] + 1] + num[1:], den, pa, pw, ex),                     # first breakpoint moved
        (num, den, pa, [pw[0] + 1] + pw[1:], ex),                      # a slope changed
    ]
    moved = ex.copy()
    i = int(np.argmax((ex > 0) & (ex <= len(bps))))
    moved[i] = ex[i] - 1 if ex[i] > 0 else ex[i] + 1
    bad.append((num, den, pa, pw, moved))                              # one exit piece changed
    for b in bad:
        with pytest.raises(AssertionError):
            check(*b)
