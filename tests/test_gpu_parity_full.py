"""Full-size parity of the HIP path with the CPU oracle.

* The benchmark workload (500x375, 25 seeds x 20 lambdas, 4- and
  8-connected): every one of the 500 solves of each connectivity is compared
  with an oracle solve, flow and minimal source set, element by element.
* The uneven workload unshrunk (256 images of 64..640 x 64..480, mixed
  connectivity, 1..16 seeds, 10..30 lambdas, about 42 000 solves in one
  call): every solve is checked by the max-flow = min-cut certificate
  (F equals the cost of the returned cut, recomputed from the original
  capacities, so both are optimal) and by nesting across lambda; the first,
  middle and last lambda of every instance are compared with oracle solves.
* All breakpoints of seeds of the benchmark workload over lambda 1..2000:
  oracle solves at both ends of the range and on both sides of every
  reported change point prove the list complete (the sets are nested in
  lambda, so equal sets at both ends of a gap leave no change inside it).
* All real breakpoints of the same seeds, proven with oracle solves at
  rational lambdas.
* The int32 headroom: n-links at the largest admitted capacity next to
  INF seeds, where excess reaches INF + K * PMF_NLINK_MAX(K).

Oracle solves run on a host thread pool while the GPU works.
"""

import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from helpers import headroom_instance, host_threads
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


def gpu_solve(pmf, insts, **opts):
    """Flows (host int64), statuses, and the solver (masks stay on the device)."""
    import torch
    opts.setdefault("max_supersteps", 2000000)
    s = pmf.Solver(**opts)
    dev = pmf.to_device(insts)
    flows, status = s.solve(dev)
    torch.cuda.synchronize()
    return flows.cpu().numpy(), status.cpu().numpy(), s, dev


def masks_of(solver, i, L):
    return np.stack([solver.extract_cut(i, k).cpu().numpy().astype(bool) for k in range(L)])


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("K", [4, 8])
def test_config2_every_solve_against_oracle(pmf, K):
    insts = W.config2(K=K)
    tasks = [(inst, int(inst.lambdas[k])) for inst in insts for k in range(inst.L)]
    threads = host_threads()
    say("config2 K=%d: %d oracle solves on %d host threads, GPU batch meanwhile" % (K, len(tasks), threads))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        fut = [ex.submit(O.fifo_pr, inst, lam) for inst, lam in tasks]
        flows, status, s, _ = gpu_solve(pmf, insts)
        assert (status == 0).all(), status
        say("gpu done; stats", s.stats())
        masks = [masks_of(s, i, inst.L) for i, inst in enumerate(insts)]
        s.close()
        j = 0
        for i, inst in enumerate(insts):
            for k in range(inst.L):
                f, m = fut[j].result()
                assert int(flows[j]) == f, ("flow", K, i, k, int(flows[j]), f)
                assert (masks[i][k] == m).all(), ("mask", K, i, k, int((masks[i][k] != m).sum()))
                j += 1
            say("instance", i, "all", inst.L, "lambdas equal")


@pytest.mark.timeout(1800)
def test_config3_full_size(pmf):
    say("generating the uneven workload (256 images)")
    insts = W.config3()
    n_solves = sum(i.L for i in insts)
    say("config3: %d instances, %d solves, sizes %s..%s, K %s" % (
        len(insts), n_solves, min(i.n for i in insts), max(i.n for i in insts), sorted({i.K for i in insts})))
    checks = []
    for i, inst in enumerate(insts):
        for k in sorted({0, inst.L // 2, inst.L - 1}):
            checks.append((i, k))
    threads = host_threads()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        fut = {c: ex.submit(O.fifo_pr, insts[c[0]], int(insts[c[0]].lambdas[c[1]])) for c in checks}
        say("%d oracle solves queued on %d threads" % (len(checks), threads))
        flows, status, s, _ = gpu_solve(pmf, insts)
        assert (status == 0).all(), np.nonzero(status)[0][:10]
        say("gpu done; stats", s.stats())
        off = np.cumsum([0] + [inst.L for inst in insts])
        cert = []
        for i, inst in enumerate(insts):
            m = masks_of(s, i, inst.L)
            for k in range(inst.L):
                if k:
                    assert not (m[k] & ~m[k - 1]).any(), ("nesting", i, k)
                cert.append((ex.submit(O.cut_cost_c, inst, int(inst.lambdas[k]), m[k]), int(flows[off[i] + k]), i, k))
            for k in sorted({0, inst.L // 2, inst.L - 1}):
                f, om = fut[(i, k)].result()
                assert int(flows[off[i] + k]) == f, ("flow", i, k, int(flows[off[i] + k]), f)
                assert (m[k] == om).all(), ("mask", i, k, int((m[k] != om).sum()))
            if i % 200 == 0:
                say("instance", i, "of", len(insts), "checked")
        s.close()
        for c, f, i, k in cert:
            assert c.result() == f, ("certificate", i, k, c.result(), f)
    say("config3: all %d solves pass the certificate and nesting, %d match the oracle" % (n_solves, len(checks)))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("K,seed", [(4, 0), (8, 12)])
def test_parametric_full_size(pmf, K, seed):
    """Every integer breakpoint in 1..2000 of one 500x375 seed instance of
    the benchmark workload, F there and each pixel's exit lambda."""
    import torch
    inst = W.config2(K=K)[seed]
    lo, hi = 1, 2000
    dev = pmf.to_device([inst])[0]
    s = pmf.Solver()
    say("parametric full size K=%d seed %d range %d..%d" % (K, seed, lo, hi))
    bp, f, ex = pmf.pmf_parametric(s.handle, dev, lo, hi)
    torch.cuda.synchronize()
    ex = ex.cpu().numpy()
    s.close()
    bp = [int(b) for b in bp]
    say("%d change points; oracle on both sides of each" % len(bp))
    assert bp == sorted(set(bp)) and all(lo < b <= hi for b in bp)
    lams = sorted({lo, hi} | {b for b in bp} | {b - 1 for b in bp})
    sols = dict(zip(lams, O.solve_many([(inst, lam) for lam in lams], threads=host_threads())))
    mask = {lam: np.asarray(m, dtype=bool).reshape(inst.H, inst.W) for lam, (_, m) in sols.items()}
    assert int(f[0]) == sols[lo][0]
    for b, fb in zip(bp, f[1:]):
        assert int(fb) == sols[b][0], ("F", b)
        assert (mask[b] != mask[b - 1]).any(), ("not a change point", b)
    # no change inside a gap: equal sets at both of its ends
    starts, ends = [lo] + bp, [b - 1 for b in bp] + [hi]
    for a, z in zip(starts, ends):
        assert (mask[a] == mask[z]).all(), ("change inside", a, z)
    exp = np.full((inst.H, inst.W), hi + 1, dtype=np.int64)
    for lam in reversed([lo] + bp):
        exp[~mask[lam]] = lam
    assert (ex == exp).all(), int((ex != exp).sum())


@pytest.mark.timeout(600)
@pytest.mark.parametrize("K,seed", [(4, 0), (8, 12)])
def test_real_breakpoints_full_size(pmf, K, seed):
    """Every real breakpoint in [1, 2000] of one 500x375 seed instance of the
    benchmark workload, proven exact with oracle solves at rational lambdas
    (each breakpoint and each piece's midpoint)."""
    import torch
    from helpers import check_breakpoints_oracle
    inst = W.config2(K=K)[seed]
    dev = pmf.to_device([inst])[0]
    s = pmf.Solver()
    say("real breakpoints full size K=%d seed %d" % (K, seed))
    num, den, pa, pw, ex = pmf.pmf_breakpoints(s.handle, dev, 1, 2000)
    torch.cuda.synchronize()
    ex = ex.cpu().numpy()
    s.close()
    say("%d breakpoints, largest denominator %d; oracle proof" % (len(num), int(den.max()) if len(den) else 1))
    check_breakpoints_oracle(inst, 1, 2000, num, den, pa, pw, ex, host_threads())


@pytest.mark.parametrize("orientation", [0, 3])
def test_int32_headroom(pmf, orientation):
    """n-links at the bound next to INF seeds: bit-exact flows (int64, about
    K * 2^30 per cut arc) and masks, in both orientations, on grids of one and
    of many tiles; a seed code outside {0, 1, 2} is rejected with EINVAL."""
    rng = np.random.default_rng(4242 + orientation)
    insts = [headroom_instance(rng, 6, 5, 4, 3), headroom_instance(rng, 7, 6, 8, 3),
             headroom_instance(rng, 70, 41, 4, 2), headroom_instance(rng, 45, 66, 8, 2)]
    bad = headroom_instance(rng, 9, 9, 4, 2)
    bad.seed = bad.seed.copy()
    bad.seed[4, 4] = 3
    say("headroom orientation", orientation, [(i.W, i.H, i.K) for i in insts])
    flows, status, s, _ = gpu_solve(pmf, insts + [bad], orientation=orientation, lambda_chunk=100)
    assert list(status) == [0, 0, 0, 0, pmf.PMF_EINVAL], status
    off = np.cumsum([0] + [i.L for i in insts + [bad]])
    assert (flows[off[4]:off[5]] == -1).all()
    for i, inst in enumerate(insts):
        m = masks_of(s, i, inst.L)
        for k in range(inst.L):
            f, om = O.fifo_pr(inst, int(inst.lambdas[k]))
            assert int(flows[off[i] + k]) == f, ("flow", i, k)
            assert (m[k] == om).all(), ("mask", i, k)
    s.close()
