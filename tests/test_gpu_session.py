"""GPU tests of the serving session (through the C ABI): instances admitted
while others run give the same results as when solved alone; slots and pool
memory are reused; a full pool refuses admission; cancellation leaves the
others intact; the serving loop returns oracle-exact results."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_06004_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1509_06004_amd import pmf
    assert torch.cuda.is_available()
    pmf.load_library()
    return torch, pmf


def alone(env, inst):
    """One instance solved by itself with pmf_solve_batch."""
    torch, pmf = env
    s = pmf.Solver(max_supersteps=400000)
    flows, status = s.solve(pmf.to_device([inst]))
    torch.cuda.synchronize()
    masks = np.stack([s.extract_cut(0, k).cpu().numpy().astype(bool) for k in range(inst.L)])
    out = flows.cpu().numpy(), int(status.cpu()[0]), masks
    s.close()
    return out


class Session:
    def __init__(self, env, slots=64, pool=0, **opts):
        torch, pmf = env
        self.torch, self.pmf = torch, pmf
        o = pmf.pmf_default_options()
        o.max_supersteps = 400000
        for k, v in opts.items():
            setattr(o, k, v)
        self.h = pmf.pmf_create(o, int(torch.cuda.current_stream().cuda_stream))
        assert pmf.pmf_session_open(self.h, slots, pool) == pmf.PMF_OK
        self.keep = {}

    def submit(self, insts):
        torch, pmf = self.torch, self.pmf
        dev = pmf.to_device(insts)
        flows = torch.full((sum(d.L for d in dev),), -7, dtype=torch.int64, device="cuda")
        status = torch.full((len(dev),), -7, dtype=torch.int32, device="cuda")
        rc, ids = pmf.pmf_session_submit(self.h, [d.c_struct() for d in dev], int(flows.data_ptr()),
                                         int(status.data_ptr()))
        if rc != pmf.PMF_OK:
            return rc, []
        off = 0
        for j, (i, d) in enumerate(zip(ids, dev)):
            self.keep[i] = (d, flows, status, off, j)
            off += d.L
        return rc, ids

    def step(self, n=8):
        rc, done = self.pmf.pmf_session_step(self.h, n)
        assert rc == self.pmf.PMF_OK
        return done

    def result(self, i):
        d, flows, status, off, j = self.keep[i]
        masks = []
        for k in range(d.L):
            m = self.torch.empty((d.H, d.W), dtype=self.torch.uint8, device="cuda")
            assert self.pmf.pmf_extract_cut(self.h, i, k, int(m.data_ptr())) == 0
            masks.append(m)
        lv = self.torch.empty((d.H, d.W), dtype=self.torch.uint8, device="cuda")
        assert self.pmf.pmf_extract_levels(self.h, i, int(lv.data_ptr())) == 0
        self.torch.cuda.synchronize()
        return (flows[off:off + d.L].cpu().numpy(), int(status[j].item()),
                np.stack([m.cpu().numpy().astype(bool) for m in masks]), lv.cpu().numpy())

    def close(self):
        self.pmf.pmf_destroy(self.h)


def mixed_instances(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        Wd, Hd = int(rng.integers(20, 150)), int(rng.integers(20, 120))
        out.append(W.tiny_random(rng, Wd, Hd, 4 if i % 2 else 8, cmax=int(rng.choice([30, 400])),
                                 L=int(rng.integers(1, 6)), p_seed=0.03, lam_max=80))
    return out


def test_join_while_running_equals_alone(env):
    a = mixed_instances(101, 6)
    b = mixed_instances(102, 5)
    say("session: 6 instances, then 5 more while running")
    S = Session(env)
    rc, ida = S.submit(a)
    assert rc == 0
    done = set(S.step(4))
    rc, idb = S.submit(b)  # joins the running launches
    assert rc == 0
    for _ in range(5000):
        done |= set(S.step(16))
        if done >= set(ida + idb):
            break
    assert done >= set(ida + idb)
    for i, inst in zip(ida + idb, a + b):
        f, st, m, lv = S.result(i)
        f0, st0, m0 = alone(env, inst)
        assert st == 0 and st0 == 0
        assert (f == f0).all() and (m == m0).all()
        for k in range(inst.L):
            assert ((lv > k) == m[k]).all()
        for k, lam in enumerate(inst.lambdas.tolist()):
            fo, mo = O.fifo_pr(inst, lam)
            assert f[k] == fo and (m[k] == mo).all()
    S.close()


def test_release_reuse_and_admission(env):
    torch, pmf = env
    insts = mixed_instances(103, 4)
    need = pmf.pmf_query_bytes([pmf.InstanceC(i.W, i.H, i.K, i.L, 1, 1, 1, 0, 0, 1) for i in insts])
    S = Session(env, slots=8, pool=need)  # room for exactly these four
    rc, ids = S.submit(insts)
    assert rc == 0
    more = mixed_instances(104, 1)
    rc2, _ = S.submit(more)
    assert rc2 == pmf.PMF_EBUSY  # pool full: nothing admitted
    info = pmf.pmf_session_query(S.h)
    assert info["running"] == 4 and info["admitted"] == 4
    done = set()
    for _ in range(5000):
        done |= set(S.step(16))
        if done >= set(ids):
            break
    first = [S.result(i) for i in ids]
    for i in ids:
        assert pmf.pmf_session_release(S.h, i) == 0
    assert pmf.pmf_session_release(S.h, ids[0]) == pmf.PMF_ERANGE
    # the same instances again, in the freed slots and memory
    rc, ids2 = S.submit(insts)
    assert rc == 0 and sorted(ids2) == sorted(ids)
    done = set()
    for _ in range(5000):
        done |= set(S.step(16))
        if done >= set(ids2):
            break
    for r0, i in zip(first, ids2):
        r1 = S.result(i)
        assert (r0[0] == r1[0]).all() and (r0[2] == r1[2]).all()
    S.close()


def test_cancel_leaves_others_intact(env):
    torch, pmf = env
    insts = mixed_instances(105, 5)
    S = Session(env)
    rc, ids = S.submit(insts)
    assert rc == 0
    S.step(2)
    victim = ids[2]
    assert pmf.pmf_session_release(S.h, victim) == 0
    keep = [i for i in ids if i != victim]
    done = set()
    for _ in range(5000):
        done |= set(S.step(16))
        if done >= set(keep):
            break
    assert victim not in done
    for i in keep:
        inst = insts[ids.index(i)]
        f, st, m, _ = S.result(i)
        f0, _, m0 = alone(env, inst)
        assert (f == f0).all() and (m == m0).all()
    S.close()


@pytest.mark.parametrize("chunk", [0, 2])
def test_serving_loop_results_exact(env, chunk):
    """Requests served through the continuous-batching loop (arrivals overlap)
    return exactly the oracle's flows and nested masks, whole warm chains
    (chunk 0) and schedules split into chunks of two lambdas alike."""
    from paper_1509_06004_amd.serve import PmfBackend, Server
    rng = np.random.default_rng(106)
    reqs = []
    for r in range(10):
        img = W.voronoi_image(int(rng.integers(40, 120)), int(rng.integers(40, 100)), 8, rng)
        K = 4 if r % 2 else 8
        nl = W.nlinks(img, K)
        H, Wd = img.shape
        reqs.append([W.seed_instance(img, nl, K, int(rng.integers(5, Wd - 5)), int(rng.integers(5, H - 5)), 5,
                                     W.loguniform_lambdas(rng, int(rng.integers(2, 6)), 300.0), image=r)
                     for _ in range(int(rng.integers(1, 4)))])
    arrivals = np.sort(rng.uniform(0, 0.2, size=len(reqs)))
    say("serving 10 requests, lambda chunk %d" % chunk)
    be = PmfBackend(max_slots=256, pool_bytes=1 << 30, supersteps=8, lambda_chunk=chunk, max_supersteps=400000)
    rep = Server(be, keep_results=True).run(arrivals, lambda i: reqs[i], duration_s=5.0, drain=True)
    be.close()
    assert rep.completed == 10 and rep.failed == 0
    for rec in rep.records:
        for inst, res in zip(reqs[rec.index], rec.results):
            assert res.status == 0
            for k, lam in enumerate(inst.lambdas.tolist()):
                f, m = O.fifo_pr(inst, lam)
                assert res.flows[k] == f
                assert ((res.levels > k) == m).all()


def test_session_after_batch_on_one_handle(env):
    """A batch solve, then a session on the same handle: the superstep graph
    the batch captured stays with the handle and must not serve the session's
    other work list.  Every session result equals the instance solved alone,
    and the batch's results equal their own solves alone."""
    torch, pmf = env
    o = pmf.pmf_default_options()
    o.max_supersteps = 400000
    h = pmf.pmf_create(o, int(torch.cuda.current_stream().cuda_stream))
    batch = mixed_instances(21, 5)
    devb = pmf.to_device(batch)
    fb = torch.full((sum(d.L for d in devb),), -7, dtype=torch.int64, device="cuda")
    sb = torch.full((len(devb),), -7, dtype=torch.int32, device="cuda")
    assert pmf.pmf_solve_batch(h, [d.c_struct() for d in devb], int(fb.data_ptr()), int(sb.data_ptr())) == 0
    torch.cuda.synchronize()
    off = 0
    for inst in batch:
        f, st, _ = alone(env, inst)
        assert st == 0 and np.array_equal(fb.cpu().numpy()[off:off + inst.L], f)
        off += inst.L
    S = Session.__new__(Session)
    S.torch, S.pmf, S.h, S.keep = torch, pmf, h, {}
    assert pmf.pmf_session_open(h, 64, 0) == pmf.PMF_OK
    insts = mixed_instances(22, 6)
    rc, ids = S.submit(insts)
    assert rc == pmf.PMF_OK
    left = set(ids)
    for _ in range(20000):
        left -= set(S.step(16))
        if not left:
            break
    assert not left
    for i, inst in zip(ids, insts):
        f, st, m, _ = S.result(i)
        fa, sa, ma = alone(env, inst)
        assert st == sa == 0 and np.array_equal(f, fa) and np.array_equal(m, ma), i
    S.close()
