"""GPU checks of the boundary's extra calls, through the C ABI: the
asynchronous solve (same results as the blocking one, the caller's thread is
free meanwhile), and all-breakpoints runs inside the handle's own memory
(a caller workspace, a memory budget)."""

import sys
import time

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


def test_async_solve_matches_blocking(pmf):
    import torch
    insts = W.config1() + W.config2(K=4, seeds=3, L=6)
    dev = pmf.to_device(insts)
    ref = pmf.Solver()
    f0, s0 = ref.solve(dev)
    torch.cuda.synchronize()
    m0 = [[ref.extract_cut(i, k).cpu() for k in range(inst.L)] for i, inst in enumerate(insts)]
    a = pmf.Solver()
    for rep in range(2):
        t0 = time.perf_counter()
        f1, s1 = a.solve_async(dev)
        t_ret = time.perf_counter() - t0
        polls = 0
        while not a.done():
            polls += 1
            time.sleep(0.0005)
        a.wait()
        t_all = time.perf_counter() - t0
        torch.cuda.synchronize()
        say("async solve", rep, "returned after %.2f ms, done after %.2f ms, %d polls" % (t_ret * 1e3, t_all * 1e3, polls))
        assert torch.equal(f0, f1) and torch.equal(s0, s1)
        for i, inst in enumerate(insts):
            for k in range(inst.L):
                assert torch.equal(m0[i][k], a.extract_cut(i, k).cpu()), (i, k)
    assert int(s1.cpu().max()) == 0
    for k in (0, 9, 19):
        f, m = O.fifo_pr(insts[0], int(insts[0].lambdas[k]))
        assert int(f1[k].cpu()) == f
    # a call on the handle while a solve is outstanding waits for it
    f2, _ = a.solve_async(dev)
    st = a.stats()
    assert st["supersteps"] > 0
    assert torch.equal(f0, f2)
    a.close()
    ref.close()


def test_parametric_in_workspace_and_budget(pmf):
    """All breakpoints inside a caller workspace give the same answer as with
    library memory; a memory budget too small is reported, not exceeded."""
    import torch
    inst = W.config0()[0]
    dev = pmf.to_device([inst])[0]
    s = pmf.Solver()
    bp0, f0, ex0 = pmf.pmf_parametric(s.handle, dev, 0, 250)
    torch.cuda.synchronize()
    s.close()
    ws = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    w = pmf.Solver(workspace=ws)
    bp1, f1, ex1 = pmf.pmf_parametric(w.handle, dev, 0, 250)
    torch.cuda.synchronize()
    assert list(bp0) == list(bp1) and list(f0) == list(f1)
    assert torch.equal(ex0, ex1)
    assert w.stats()["device_bytes"] <= ws.numel()
    w.close()
    small = pmf.Solver(mem_budget=1 << 16)
    with pytest.raises(pmf.PmfError) as e:
        pmf.pmf_parametric(small.handle, dev, 0, 250)
    assert e.value.code == pmf.PMF_ENOMEM
    small.close()
    # and the breakpoints themselves against the oracle at every integer lambda
    lams = list(range(0, 251))
    sols = O.solve_many([(inst, lam) for lam in lams])
    ms = np.stack([np.asarray(m, dtype=bool).reshape(inst.H, inst.W) for _, m in sols])
    exp_bp = [lams[i] for i in range(1, len(lams)) if (ms[i] != ms[i - 1]).any()]
    assert list(bp1) == exp_bp


def test_pixel_visit_statistics(pmf):
    """Visit statistics: with an orientation count every instance (chunk) is
    counted and initialised exactly once, so both totals are its pixels; the
    per-kind counts of timing mode equal the instances' own counters."""
    import torch
    insts = W.config1() + W.config2(K=4, seeds=2, L=5) + W.config2(K=8, seeds=1, L=4)
    dev = pmf.to_device(insts)
    chunk = 2
    px = sum(inst.W * inst.H * ((inst.L + chunk - 1) // chunk) for inst in insts)
    px_all_lambdas = sum(inst.W * inst.H * inst.L for inst in insts)
    for timing in (0, 1):
        s = pmf.Solver(lambda_chunk=chunk, orientation=2, timing=timing)
        s.solve(dev)
        torch.cuda.synchronize()
        st = s.stats()
        say("timing", timing, {k: st[k] for k in ("px_orient", "px_init", "px_init_x", "px_sweep", "px_relabel", "px_cut")})
        assert st["px_orient"] == px
        assert st["px_init"] + st["px_init_x"] == px
        # every lambda's cut starts with a pass over all of the instance's tiles
        assert st["px_relabel"] > 0 and st["px_cut"] + st["px_cut_x"] >= px_all_lambdas
        if timing:
            kp = st["kernel_px"]
            own = [st["px_sweep"], st["px_relabel"], st["px_cut"], st["px_init"], st["px_orient"],
                   st["px_init_x"], st["px_cut_x"]]
            assert [int(kp[i]) + int(kp[8 + i]) for i in range(7)] == own


def test_same_shape_batches_on_one_handle(pmf):
    """Consecutive batches of the same shape on one handle (the captured
    superstep graph is replayed for the second, with new descriptors and
    states): each batch equals the oracle, element by element."""
    import torch
    s = pmf.Solver()
    for seed in (11, 12):
        rng = np.random.default_rng(seed)
        insts = [W.tiny_random(rng, 70, 50, K, cmax=40, L=4, lam_max=40) for K in (4, 4, 8)]
        dev = pmf.to_device(insts)
        flows, status = s.solve(dev)
        torch.cuda.synchronize()
        assert int(status.cpu().max()) == 0
        f = flows.cpu().numpy()
        off = 0
        for i, inst in enumerate(insts):
            for k in range(inst.L):
                fo, mo = O.fifo_pr(inst, int(inst.lambdas[k]))
                assert int(f[off + k]) == fo, (seed, i, k)
                got = s.extract_cut(i, k).cpu().numpy().astype(bool)
                assert np.array_equal(got, np.asarray(mo, dtype=bool).reshape(inst.H, inst.W)), (seed, i, k)
            off += inst.L
        say("batch", seed, "equals the oracle; supersteps", s.stats()["supersteps"])


def _two_pixel_instance(nl_cap):
    """Two free pixels joined both ways by n-links of capacity nl_cap, source
    capacity 5 each, sink slopes 1 and 2: while nl_cap binds them, F is
    min(10, 3 lambda) with its only breakpoint at 10/3."""
    nl = np.zeros((4, 1, 2), dtype=np.int32)
    nl[0, 0, 0] = nl_cap  # (0,0) -> (1,0)
    nl[1, 0, 1] = nl_cap  # (1,0) -> (0,0)
    return W.Instance(W=2, H=1, K=4, nlink=nl, cap_src=np.full((1, 2), 5, dtype=np.int32),
                      cap_snk0=np.zeros((1, 2), dtype=np.int32), snk_slope=np.array([[1, 2]], dtype=np.int32),
                      seed=np.zeros((1, 2), dtype=np.uint8), lambdas=np.array([0], dtype=np.int32))


def test_breakpoints_edge_cases(pmf):
    """pmf_breakpoints: a range of one lambda, a range without change, a list
    longer than max_bp (PMF_ERANGE), a probe whose scaled capacities would
    leave int32 (PMF_ERANGE rather than an inexact answer), and the same
    answer in a caller workspace as in library memory, with a budget too
    small reported as PMF_ENOMEM."""
    import torch
    from fractions import Fraction
    s = pmf.Solver()
    inst = _two_pixel_instance(100)
    dev = pmf.to_device([inst])[0]
    num, den, pa, pw, ex = pmf.pmf_breakpoints(s.handle, dev, 0, 10)
    assert [Fraction(int(a), int(b)) for a, b in zip(num, den)] == [Fraction(10, 3)]
    assert list(pa) == [0, 10] and list(pw) == [3, 0]
    assert (ex.cpu().numpy() == 1).all()  # both pixels leave at the one breakpoint
    # one lambda (both pixels stay: exit piece 1 = never leaves), and a range
    # with no change (neither pixel is ever in S_min: exit piece 0)
    for lo, hi, a, w, e in ((2, 2, 0, 3, 1), (5, 9, 10, 0, 0)):
        num, den, pa, pw, ex = pmf.pmf_breakpoints(s.handle, dev, lo, hi)
        assert len(num) == 0 and list(pa) == [a] and list(pw) == [w], (lo, hi)
        assert (ex.cpu().numpy() == e).all(), (lo, hi)
    # more breakpoints than max_bp
    big = W.config0()[0]
    bdev = pmf.to_device([big])[0]
    num, den, pa, pw, ex = pmf.pmf_breakpoints(s.handle, bdev, 0, 250)
    assert len(num) >= 2
    with pytest.raises(pmf.PmfError) as e:
        pmf.pmf_breakpoints(s.handle, bdev, 0, 250, max_bp=1)
    assert e.value.code == pmf.PMF_ERANGE
    # n-links so large that 3 times them leave the solver's bound
    hdev = pmf.to_device([_two_pixel_instance(((1 << 30) - 1) // 4)])[0]  # PMF_NLINK_MAX(4)
    with pytest.raises(pmf.PmfError) as e:
        pmf.pmf_breakpoints(s.handle, hdev, 0, 10)
    assert e.value.code == pmf.PMF_ERANGE
    s.close()
    # a caller workspace gives the same answer; a budget too small is reported
    ws = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    w = pmf.Solver(workspace=ws)
    num1, den1, pa1, pw1, ex1 = pmf.pmf_breakpoints(w.handle, bdev, 0, 250)
    torch.cuda.synchronize()
    assert list(num1) == list(num) and list(den1) == list(den)
    assert list(pa1) == list(pa) and list(pw1) == list(pw) and torch.equal(ex1, ex)
    w.close()
    small = pmf.Solver(mem_budget=1 << 16)
    with pytest.raises(pmf.PmfError) as e:
        pmf.pmf_breakpoints(small.handle, bdev, 0, 250)
    assert e.value.code == pmf.PMF_ENOMEM
    small.close()


def test_breakpoints_do_not_depend_on_options(pmf):
    """The real breakpoints, piece lines and exit pieces are the same under
    every speed option that changes how the probes are solved: tile shape,
    orientation policy, gap heuristic, persistent launch, timing mode."""
    rng = np.random.default_rng(79)
    cases = [(W.config0()[0], 0, 250),
             (W.tiny_random(rng, 16, 13, 8, cmax=200, L=1, p_seed=0.05), 2, 600)]
    variants = [{}, {"tile_w": 64, "tile_h": 16}, {"orientation": 0}, {"orientation": 3}, {"gap": 1},
                {"persist_tiles": 1 << 20}, {"timing": 2}]
    for ci, (inst, lo, hi) in enumerate(cases):
        dev = pmf.to_device([inst])[0]
        ref = None
        for opts in variants:
            s = pmf.Solver(**opts)
            num, den, pa, pw, ex = pmf.pmf_breakpoints(s.handle, dev, lo, hi)
            got = (list(num), list(den), list(pa), list(pw), ex.cpu().numpy())
            s.close()
            say("breakpoints case", ci, "options", opts, "breakpoints", len(num))
            if ref is None:
                ref = got
                assert len(num) >= 3, ci
                continue
            assert got[:4] == ref[:4], (ci, opts)
            assert (got[4] == ref[4]).all(), (ci, opts)
