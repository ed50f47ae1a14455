"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Flows (int64) and minimal source-side masks must be bit-exact.  The oracle
solves every lambda from scratch; the GPU continues each schedule from the
previous lambda's preflow, so agreement also checks the warm start.
"""

import sys

from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_06004_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pmf():
    import torch
    from paper_1509_06004_amd import pmf as P
    assert torch.cuda.is_available()
    P.load_library()
    return P


def solve(pmf, insts, **opts):
    import torch
    opts.setdefault("max_supersteps", 400000)
    s = pmf.Solver(**opts)
    dev = pmf.to_device(insts)
    flows, status = s.solve(dev)
    torch.cuda.synchronize()
    masks = []
    st = status.cpu().numpy()
    for i, inst in enumerate(insts):
        if st[i] != 0:  # no masks for an instance that failed validation
            masks.append(None)
            continue
        masks.append(np.stack([s.extract_cut(i, k).cpu().numpy().astype(bool) for k in range(inst.L)]))
    out = (flows.cpu().numpy(), st, masks, s.stats())
    s.close()
    return out


def split(flows, insts):
    out, o = [], 0
    for inst in insts:
        out.append(flows[o:o + inst.L])
        o += inst.L
    return out


def check_against_oracle(insts, flows, status, masks, lam_idx=None):
    fl = split(flows, insts)
    for i, inst in enumerate(insts):
        assert status[i] == 0, (i, status[i])
        ks = range(inst.L) if lam_idx is None else lam_idx(i, inst)
        for k in ks:
            lam = int(inst.lambdas[k])
            f, m = O.fifo_pr(inst, lam)
            assert fl[i][k] == f, ("flow", i, k, lam, fl[i][k], f)
            assert (masks[i][k] == m).all(), ("mask", i, k, lam, int((masks[i][k] != m).sum()))


def test_golden_fixtures(pmf):
    from helpers import golden_instances
    gold = golden_instances()
    say("golden fixtures", len(gold))
    insts = [g[1] for g in gold]
    flows, status, masks, _ = solve(pmf, insts)
    for i, (name, inst, fl, ms) in enumerate(gold):
        assert status[i] == 0
        assert list(split(flows, insts)[i]) == list(fl), name
        assert (masks[i] == ms).all(), name


def test_tiny_random_batch(pmf):
    """Many tiny grids (all shapes up to 9x9, 4/8-conn, seeds, INF arcs, ties) in one batch."""
    rng = np.random.default_rng(7)
    insts = []
    for i in range(160):
        Wd, Hd = int(rng.integers(1, 10)), int(rng.integers(1, 10))
        cmax = int(rng.choice([1, 3, 20, 500]))
        insts.append(W.tiny_random(rng, Wd, Hd, 4 if i % 2 else 8, cmax=cmax, L=int(rng.integers(1, 5)),
                                   p_seed=float(rng.uniform(0, 0.3)), lam_max=3 * cmax,
                                   p_inf_nlink=0.1 if i % 7 == 0 else 0.0))
    say("tiny batch", len(insts))
    flows, status, masks, _ = solve(pmf, insts)
    check_against_oracle(insts, flows, status, masks)


@pytest.mark.parametrize("orientation,chunk", [(3, 0), (3, 100), (1, 1), (2, 100)])
def test_orientation_edge_cases(pmf, orientation, chunk):
    """Solving with source and sink exchanged (always, or by either counting
    rule; warm chains included) gives the oracle's flows and minimal source
    sets on the golden fixtures and on tiny grids with seeds, INF n-links and
    ties."""
    from helpers import golden_instances
    gold = golden_instances()
    insts = [g[1] for g in gold]
    flows, status, masks, _ = solve(pmf, insts, orientation=orientation, lambda_chunk=chunk)
    for i, (name, inst, fl, ms) in enumerate(gold):
        assert status[i] == 0
        assert list(split(flows, insts)[i]) == list(fl), name
        assert (masks[i] == ms).all(), name
    rng = np.random.default_rng(71 + orientation)
    tiny = []
    for i in range(80):
        Wd, Hd = int(rng.integers(1, 10)), int(rng.integers(1, 10))
        cmax = int(rng.choice([1, 3, 20, 500]))
        tiny.append(W.tiny_random(rng, Wd, Hd, 4 if i % 2 else 8, cmax=cmax, L=int(rng.integers(1, 5)),
                                  p_seed=float(rng.uniform(0, 0.3)), lam_max=3 * cmax,
                                  p_inf_nlink=0.1 if i % 7 == 0 else 0.0))
    say("orientation", orientation, "chunk", chunk, "tiny", len(tiny))
    flows, status, masks, _ = solve(pmf, tiny, orientation=orientation, lambda_chunk=chunk)
    check_against_oracle(tiny, flows, status, masks)


@pytest.mark.parametrize("K,xsw", [(4, 4), (8, 2)])
def test_sweep_exchanges_repeated(pmf, K, xsw):
    """Sweep visits that hand flow to running neighbour tiles and take theirs
    during the visit (every superstep counted as short): warm chains on grids
    of many tiles, both orientations, three solves, oracle-exact."""
    rng = np.random.default_rng(800 + K)
    insts = []
    for i in range(4):
        img = W.voronoi_image(int(rng.integers(70, 140)), int(rng.integers(60, 110)), 8, rng)
        nl = W.nlinks(img, K)
        H, Wd = img.shape
        insts.append(W.seed_instance(img, nl, K, int(rng.integers(5, Wd - 5)), int(rng.integers(5, H - 5)), 5,
                                     W.loguniform_lambdas(rng, 6, 2000.0), image=i))
    for rep in range(3):
        say("sweep exchanges K", K, "xsw", xsw, "solve", rep)
        flows, status, masks, _ = solve(pmf, insts, tail_tiles=1 << 30, tail_sweep_exchanges=xsw,
                                        orientation=2 if rep else 0, lambda_chunk=100 if rep < 2 else 2)
        check_against_oracle(insts, flows, status, masks)


@pytest.mark.parametrize("K", [4, 8])
def test_warm_chains_as_given_repeated(pmf, K):
    """Whole warm chains solved as given (never exchanged), on grids of many
    tiles: three solves of the same batch each match the oracle at every
    lambda (a race between tiles would surface as a wrong flow in some run)."""
    rng = np.random.default_rng(300 + K)
    insts = []
    for i in range(4):
        img = W.voronoi_image(int(rng.integers(70, 130)), int(rng.integers(60, 110)), 8, rng)
        nl = W.nlinks(img, K)
        H, Wd = img.shape
        insts.append(W.seed_instance(img, nl, K, int(rng.integers(5, Wd - 5)), int(rng.integers(5, H - 5)), 5,
                                     W.loguniform_lambdas(rng, 8, 400.0), image=i))
    for rep in range(3):
        say("warm chains as given K", K, "solve", rep)
        flows, status, masks, _ = solve(pmf, insts, orientation=0, lambda_chunk=100)
        check_against_oracle(insts, flows, status, masks)


@pytest.mark.parametrize("orientation", [0, 2])
def test_gap_heuristic(pmf, orientation):
    """The gap heuristic (a label histogram per instance; pixels above an
    emptied level stop until the next global relabel) leaves every flow and
    minimal source set equal to the oracle's, on warm chains over grids of
    many tiles with long sweep periods (so that levels empty between
    relabels), and it does stop pixels on them."""
    rng = np.random.default_rng(900 + orientation)
    insts = []
    for i in range(6):
        K = 4 if i % 2 else 8
        img = W.voronoi_image(int(rng.integers(70, 160)), int(rng.integers(60, 120)), 10, rng)
        nl = W.nlinks(img, K)
        H, Wd = img.shape
        insts.append(W.seed_instance(img, nl, K, int(rng.integers(5, Wd - 5)), int(rng.integers(5, H - 5)), 5,
                                     W.loguniform_lambdas(rng, 6, 2000.0), image=i))
    kills = 0
    for opts in (dict(), dict(sweeps_per_relabel=64, inner_iters=4), dict(lambda_chunk=1)):
        say("gap heuristic orientation", orientation, opts)
        flows, status, masks, st = solve(pmf, insts, gap=1, orientation=orientation,
                                         **dict(dict(lambda_chunk=100), **opts))
        say("gap kills", st["gap_kills"])
        kills += st["gap_kills"]
        check_against_oracle(insts, flows, status, masks)
    assert kills > 0


@pytest.mark.parametrize("K,orientation,wgs", [(4, 2, 0), (8, 0, 16), (4, 0, 0)])
def test_persistent_supersteps(pmf, K, orientation, wgs):
    """Supersteps run back to back inside one cooperative launch (grid-wide
    barriers between compaction, tile work and the phase machine) once the
    lists are short: every flow and minimal source set equals the oracle's,
    in three repeated solves of warm chains on grids of many tiles and on a
    batch of tiny grids, and the persistent launch does run."""
    rng = np.random.default_rng(500 + K + orientation)
    insts = []
    for i in range(4):
        img = W.voronoi_image(int(rng.integers(70, 150)), int(rng.integers(60, 120)), 8, rng)
        nl = W.nlinks(img, K)
        H, Wd = img.shape
        insts.append(W.seed_instance(img, nl, K, int(rng.integers(5, Wd - 5)), int(rng.integers(5, H - 5)), 5,
                                     W.loguniform_lambdas(rng, 6, 2000.0), image=i))
    for i in range(40):
        Wd, Hd = int(rng.integers(1, 10)), int(rng.integers(1, 10))
        cmax = int(rng.choice([1, 3, 20, 500]))
        insts.append(W.tiny_random(rng, Wd, Hd, 4 if i % 2 else 8, cmax=cmax, L=int(rng.integers(1, 5)),
                                   p_seed=float(rng.uniform(0, 0.3)), lam_max=3 * cmax))
    for rep in range(3):
        say("persistent K", K, "orientation", orientation, "wgs", wgs, "solve", rep)
        flows, status, masks, st = solve(pmf, insts, persist_tiles=1 << 20, persist_wgs=wgs, steps_per_sync=4,
                                         orientation=orientation, lambda_chunk=100 if rep < 2 else 2)
        say("persistent launches", st["persist_launches"], "supersteps", st["persist_supersteps"], "of",
            st["supersteps"])
        assert st["persist_launches"] > 0 and st["persist_supersteps"] > 0
        check_against_oracle(insts, flows, status, masks)


def test_config0(pmf):
    insts = W.config0()
    say("config0 64x64")
    flows, status, masks, st = solve(pmf, insts)
    say("stats", st)
    check_against_oracle(insts, flows, status, masks)


@pytest.mark.parametrize("tile_w", [64, 32])
def test_ragged_midsize(pmf, tile_w):
    """Sizes that are not multiples of any tile, several tiles per instance."""
    rng = np.random.default_rng(17 + tile_w)
    insts = []
    for i, (Wd, Hd) in enumerate([(70, 19), (33, 65), (129, 40), (1, 77), (90, 1), (65, 33)]):
        insts.append(W.tiny_random(rng, Wd, Hd, 8 if i % 2 else 4, cmax=int(rng.choice([5, 60, 900])),
                                   L=3, p_seed=0.05, lam_max=60))
    say("ragged midsize tile_w", tile_w)
    flows, status, masks, _ = solve(pmf, insts, tile_w=tile_w, tile_h=1024 // tile_w)
    check_against_oracle(insts, flows, status, masks)


def test_config1_warm_chain(pmf):
    insts = W.config1()
    say("config1 320x240 x 20 lambdas")
    flows, status, masks, st = solve(pmf, insts)
    say("stats", st)
    check_against_oracle(insts, flows, status, masks)


def test_options_do_not_change_results(pmf):
    """Tile shape, inner iterations, relabel period, packing order, graph replay,
    lambda chunks, exchange rounds, tail settings, orientation (s-t swap):
    speed knobs only; results are identical."""
    rng = np.random.default_rng(29)
    insts = [W.tiny_random(rng, 90, 70, 4, cmax=300, L=4, p_seed=0.02, lam_max=100),
             W.tiny_random(rng, 61, 83, 8, cmax=300, L=3, p_seed=0.02, lam_max=100)]
    ref = None
    for opts in [dict(), dict(tile_w=64, tile_h=16), dict(inner_iters=1, sweeps_per_relabel=1),
                 dict(inner_iters=64, sweeps_per_relabel=32, local_bfs_iters=4), dict(order=0),
                 dict(use_graph=0, steps_per_sync=3), dict(timing=1), dict(timing=2), dict(lambda_chunk=1),
                 dict(lambda_chunk=3), dict(lambda_chunk=100), dict(exchange_rounds=1),
                 dict(exchange_rounds=16, local_bfs_iters=2), dict(tail_tiles=0),
                 dict(tail_tiles=1 << 30, tail_inner_iters=3, tail_exchange_rounds=1),
                 dict(tail_tiles=1 << 30, tail_inner_iters=200, tail_exchange_rounds=64),
                 dict(relabel_passes=1), dict(relabel_passes=2, exchange_rounds=1, local_bfs_iters=3),
                 dict(orientation=1), dict(orientation=2), dict(orientation=3),
                 dict(orientation=3, lambda_chunk=100), dict(orientation=2, lambda_chunk=2),
                 dict(gap=1), dict(gap=1, orientation=0, lambda_chunk=100),
                 dict(gap=1, inner_iters=64, sweeps_per_relabel=32, relabel_passes=2),
                 dict(persist_tiles=1 << 30), dict(persist_tiles=1 << 30, persist_wgs=8, steps_per_sync=3),
                 dict(persist_tiles=40, gap=1, lambda_chunk=1),
                 dict(tail_sweep_exchanges=3), dict(tail_tiles=1 << 30, tail_sweep_exchanges=5, tail_inner_iters=24),
                 dict(tail_tiles=1 << 30, tail_sweep_exchanges=64, tail_inner_iters=8, orientation=0)]:
        say("options", opts)
        flows, status, masks, _ = solve(pmf, insts, **opts)
        assert (status == 0).all()
        got = (flows, [m.copy() for m in masks])
        if ref is None:
            ref = got
            check_against_oracle(insts, flows, status, masks)
        else:
            assert (got[0] == ref[0]).all()
            assert all((a == b).all() for a, b in zip(got[1], ref[1]))


def test_config2_full_size_sampled(pmf):
    """The benchmark workload at full size (500x375, 4- and 8-connected, 25 seeds
    x 20 lambdas, one batched call): oracle-exact on a sample of solves, and
    every solve checked by the flow = cut-cost certificate and by nesting."""
    for K in (4, 8):
        insts = W.config2(K=K)
        say("config2 full size K=%d" % K)
        flows, status, masks, st = solve(pmf, insts)
        say("stats", st)
        fl = split(flows, insts)
        assert (status == 0).all()
        for i, inst in enumerate(insts):
            for k in range(inst.L):
                assert O.cut_cost_c(inst, int(inst.lambdas[k]), masks[i][k]) == fl[i][k]
                if k:
                    assert not (masks[i][k] & ~masks[i][k - 1]).any()
        picks = [(0, 0), (7, 3), (12, 9), (18, 14), (24, 19)] if K == 4 else [(3, 1), (21, 8)]
        for i, k in picks:
            f, m = O.fifo_pr(insts[i], int(insts[i].lambdas[k]))
            assert fl[i][k] == f and (masks[i][k] == m).all(), (K, i, k)


def test_config3_uneven_subset(pmf):
    """Uneven sizes and mixed connectivity in one call (images of the uneven
    workload, shrunk so the oracle check stays short), bit-exact."""
    insts = []
    for img in range(6):
        rng = W.rng_for(3, img)
        insts.extend(W.random_image_instances(rng, img, 64, 200, 64, 160, 3))
    say("config3-like subset", len(insts), sorted({(i.W, i.H, i.K) for i in insts}))
    flows, status, masks, _ = solve(pmf, insts)
    check_against_oracle(insts, flows, status, masks,
                         lam_idx=lambda i, inst: sorted({0, inst.L // 2, inst.L - 1}))


def test_invalid_capacities_report_status(pmf):
    """Bad values are found on the device: that instance gets EINVAL/EOVERFLOW
    and flows -1; the other instances of the batch are unaffected."""
    rng = np.random.default_rng(31)
    good = W.tiny_random(rng, 20, 15, 4, cmax=20, L=2)
    neg = W.tiny_random(rng, 20, 15, 4, cmax=20, L=2)
    neg.cap_src[3, 4] = -1
    offgrid = W.tiny_random(rng, 20, 15, 4, cmax=20, L=2)
    offgrid.nlink[0, 2, 19] = 5  # arc towards x = 20, off the grid
    over = W.tiny_random(rng, 20, 15, 8, cmax=20, L=2)
    over.nlink[1, 5, 5] = (1 << 30)  # beyond the int32 headroom for K = 8
    sink = W.tiny_random(rng, 20, 15, 4, cmax=20, L=2)
    sink.snk_slope[:] = 1
    sink.lambdas[:] = [5, 1 << 30]  # cap_snk0 + slope * lambda > INF
    badlam = W.tiny_random(rng, 20, 15, 4, cmax=20, L=2)
    badlam.lambdas[:] = [9, 3]  # decreasing schedule
    insts = [good, neg, offgrid, over, sink, badlam]
    # the decreasing pair of badlam straddles two chunks when chunk = 1
    for chunk, orientation in ((1, 0), (2, 0), (1, 3), (2, 1)):
        flows, status, masks, _ = solve(pmf, insts, lambda_chunk=chunk, orientation=orientation)
        fl = split(flows, insts)
        assert list(status) == [0, pmf.PMF_EINVAL, pmf.PMF_EINVAL, pmf.PMF_EOVERFLOW, pmf.PMF_EOVERFLOW,
                                pmf.PMF_EINVAL], chunk
        for i in range(1, len(insts)):
            assert (fl[i] == -1).all()
        check_against_oracle([good], fl[0], status[:1], masks[:1])


def test_superstep_budget_times_out(pmf):
    """A budget too small to finish (forced from the host): status ETIMEOUT,
    flows of unfinished lambdas -1, and every kernel still exits normally."""
    import torch
    insts = W.config1()
    s = pmf.Solver(max_supersteps=40, lambda_chunk=20)  # one warm chain: finished lambdas form a prefix
    flows, status = s.solve(pmf.to_device(insts))
    torch.cuda.synchronize()
    assert int(status.cpu()[0]) == pmf.PMF_ETIMEOUT
    f = flows.cpu().numpy()
    assert f[-1] == -1
    done = int((f >= 0).sum())
    for k in range(done):
        assert f[k] == O.fifo_pr(insts[0], int(insts[0].lambdas[k]))[0]
    assert (f[done:] == -1).all()
    s.close()
    s = pmf.Solver(max_supersteps=12, lambda_chunk=1)  # every lambda on its own budget
    flows, status = s.solve(pmf.to_device(insts))
    torch.cuda.synchronize()
    f = flows.cpu().numpy()
    assert int(status.cpu()[0]) == pmf.PMF_ETIMEOUT and (f == -1).any()
    for k in range(len(f)):
        assert f[k] == -1 or f[k] == O.fifo_pr(insts[0], int(insts[0].lambdas[k]))[0]
    s.close()


def test_slot_stats_describe_the_split(pmf):
    """Per-slot counters: with every lambda in its own chunk, config 1 uses 20
    slots, each finished with one lambda done and positive work counters."""
    import torch
    insts = W.config1()
    s = pmf.Solver(lambda_chunk=1, max_supersteps=400000)
    s.solve(pmf.to_device(insts))
    torch.cuda.synchronize()
    st = pmf.pmf_slot_stats(s.handle)
    assert st.shape == (20, 8)
    assert (st[:, 0] == 1).all() and (st[:, 5] == 1).all()
    assert (st[:, 1] > 0).all() and (st[:, 4] >= 4).all()  # >= 2 relabel + 2 cut passes
    s.close()


def test_timing_trace_matches_stats(pmf):
    """Timing modes record one trace row per superstep; its kernel times add up
    to the counters, and the results equal those of the default mode.  Mode 2
    (sweeps and passes launched apart) splits the tile-work time."""
    import torch
    insts = W.config0()
    dev = pmf.to_device(insts)
    ref = pmf.Solver()
    f0, s0 = ref.solve(dev)
    assert len(pmf.pmf_get_trace(ref.handle)) == 0
    for mode in (1, 2):
        t = pmf.Solver(timing=mode)
        f1, s1 = t.solve(dev)
        torch.cuda.synchronize()
        assert torch.equal(f0, f1) and torch.equal(s0, s1)
        tr = pmf.pmf_get_trace(t.handle)
        st = t.stats()
        assert tr.shape == (st["supersteps"], pmf.PMF_TRACE_COLS)
        assert tr[:, 7].sum() == st["work_ns"] > 0 and tr[:, 6].sum() == st["control_ns"]
        assert tr[:, 4].sum() == st["sweep_ns"] and tr[:, 5].sum() == st["pass_ns"]
        if mode == 1:
            assert st["sweep_ns"] == 0 and st["pass_ns"] == 0
        else:
            assert st["sweep_ns"] > 0 and st["pass_ns"] > 0 and st["sweep_ns"] + st["pass_ns"] == st["work_ns"]
        assert (tr[:, :4] >= 0).all() and tr[:, 0].sum() > 0 and tr[:, 2].sum() > 0
        t.close()
    ref.close()


def test_parametric_breakpoints(pmf):
    """All breakpoints of an instance over an integer lambda range equal the
    oracle's: the lambdas at which the minimal source set changes, F at each,
    and every pixel's exit lambda, all derived from oracle solves at every
    integer lambda of the range (free pixels with sink slope 0 included)."""
    rng = np.random.default_rng(97)
    cases = []
    for i in range(10):
        Wd, Hd = int(rng.integers(2, 12)), int(rng.integers(2, 12))
        inst = W.tiny_random(rng, Wd, Hd, 4 if i % 2 else 8, cmax=40, L=1, p_seed=0.1)
        cases.append((inst, int(rng.integers(0, 5)), int(rng.integers(20, 90))))
    # ranges wider than one round's probes: the meeting-point pair and the
    # spread probes decide which intervals stay open
    rng2 = np.random.default_rng(98)
    for i in range(6):
        Wd, Hd = int(rng2.integers(3, 17)), int(rng2.integers(3, 17))
        inst = W.tiny_random(rng2, Wd, Hd, 4 if i % 2 else 8, cmax=200, L=1, p_seed=0.05)
        cases.append((inst, int(rng2.integers(0, 5)), int(rng2.integers(300, 900))))
    cases.append((W.config0()[0], 0, 250))
    s = pmf.Solver()
    for ci, (inst, lo, hi) in enumerate(cases):
        lams = list(range(lo, hi + 1))
        sols = O.solve_many([(inst, lam) for lam in lams])
        fs = [int(f) for f, _ in sols]
        ms = np.stack([np.asarray(m, dtype=bool).reshape(inst.H, inst.W) for _, m in sols])
        exp_bp = [lams[i] for i in range(1, len(lams)) if (ms[i] != ms[i - 1]).any()]
        out = ~ms  # first lambda whose set lacks the pixel
        exp_exit = np.where(out.any(axis=0), np.array(lams)[out.argmax(axis=0)], hi + 1)
        dev = pmf.to_device([inst])[0]
        say("parametric case", ci, inst.W, inst.H, inst.K, "range", lo, hi, "breakpoints", len(exp_bp))
        bp, f, ex = pmf.pmf_parametric(s.handle, dev, lo, hi)
        assert list(bp) == exp_bp, ci
        assert int(f[0]) == fs[0], ci
        assert [int(x) for x in f[1:]] == [fs[b - lo] for b in exp_bp], ci
        assert (ex.cpu().numpy() == exp_exit).all(), ci
    s.close()


def test_breakpoints_exact_enumeration(pmf):
    """Every real breakpoint of grids of at most 12 pixels equals the lower
    envelope of the lines of all their source sets, in exact rational
    arithmetic: the breakpoints, each piece's line and each pixel's exit piece."""
    from helpers import envelope, source_set_lines
    rng = np.random.default_rng(1509)
    s = pmf.Solver()
    nbps = 0
    for ci in range(48):
        while True:
            Wd, Hd = int(rng.integers(1, 5)), int(rng.integers(1, 5))
            if Wd * Hd <= 12:
                break
        inst = W.tiny_random(rng, Wd, Hd, 4 if ci % 2 else 8, cmax=int(rng.choice([5, 20, 60])), L=1,
                             p_seed=float(rng.uniform(0, 0.2)))
        lo, hi = int(rng.integers(0, 4)), int(rng.integers(20, 120))
        sets, A, w = source_set_lines(inst)
        bps, pieces, psets = envelope(sets, A, w, lo, hi)
        dev = pmf.to_device([inst])[0]
        say("breakpoints enumeration case", ci, Wd, Hd, inst.K, "range", lo, hi, "breakpoints", len(bps))
        num, den, pa, pw, ex = pmf.pmf_breakpoints(s.handle, dev, lo, hi)
        got = [Fraction(int(a), int(b)) for a, b in zip(num, den)]
        assert got == bps, (ci, got, bps)
        assert [(int(a), int(b)) for a, b in zip(pa, pw)] == [(int(a), int(b)) for a, b in pieces], ci
        exm = ex.cpu().numpy().reshape(-1)
        for j, ps in enumerate(psets):
            assert ((exm > j) == ps).all(), (ci, j)
        nbps += len(bps)
    assert nbps >= 20
    s.close()


def test_breakpoints_against_rational_oracle(pmf):
    """Real breakpoints of larger grids proven exact with oracle solves at
    rational lambdas (F on the pieces' lines at both ends of every piece and
    the minimal sets inside and at the ends of every piece), including wide
    ranges whose unit intervals hold several breakpoints."""
    from helpers import check_breakpoints_oracle, host_threads
    rng = np.random.default_rng(1510)
    cases = []
    for i in range(4):
        Wd, Hd = int(rng.integers(6, 20)), int(rng.integers(6, 20))
        inst = W.tiny_random(rng, Wd, Hd, 4 if i % 2 else 8, cmax=200, L=1, p_seed=0.05)
        cases.append((inst, int(rng.integers(0, 5)), int(rng.integers(300, 700))))
    cases.append((W.config0()[0], 0, 250))
    s = pmf.Solver()
    for ci, (inst, lo, hi) in enumerate(cases):
        dev = pmf.to_device([inst])[0]
        num, den, pa, pw, ex = pmf.pmf_breakpoints(s.handle, dev, lo, hi)
        say("breakpoints oracle case", ci, inst.W, inst.H, inst.K, "range", lo, hi, "breakpoints", len(num),
            "largest denominator", int(den.max()) if len(den) else 1)
        check_breakpoints_oracle(inst, lo, hi, num, den, pa, pw, ex.cpu().numpy(), host_threads())
    s.close()


def test_breakpoints_agree_with_integer_search(pmf):
    """The two searches describe the same function: the integer change points
    are the ceilings of the real breakpoints, F at each of them lies on the
    piece that holds it, and each pixel's integer exit lambda is the ceiling
    of its real exit breakpoint (lam_lo and lam_hi + 1 for pixels never in,
    or never leaving, the minimal set)."""
    import math
    rng = np.random.default_rng(2718)
    cases = [(W.config0()[0], 0, 250), (W.tiny_random(rng, 14, 11, 4, cmax=200, L=1, p_seed=0.05), 1, 700)]
    s = pmf.Solver()
    for ci, (inst, lo, hi) in enumerate(cases):
        dev = pmf.to_device([inst])[0]
        bp, f, ex_i = pmf.pmf_parametric(s.handle, dev, lo, hi)
        num, den, pa, pw, ex_r = pmf.pmf_breakpoints(s.handle, dev, lo, hi)
        xs = [Fraction(int(a), int(b)) for a, b in zip(num, den)]
        say("integer vs real case", ci, "change points", len(bp), "breakpoints", len(xs))
        assert sorted({math.ceil(x) for x in xs}) == [int(c) for c in bp], ci
        # F at lam_lo and at each change point c, on the piece holding c
        for c, fc in zip([lo] + [int(c) for c in bp], f):
            j = sum(1 for x in xs if x <= c)
            assert int(fc) == int(pa[j]) + int(pw[j]) * c, (ci, c)
        exi, exr = ex_i.cpu().numpy(), ex_r.cpu().numpy()
        ceil_of = np.array([lo] + [math.ceil(x) for x in xs] + [hi + 1], dtype=np.int64)
        assert (ceil_of[exr] == exi).all(), ci
    s.close()
