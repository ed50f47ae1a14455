"""The entry point that allocates nothing (pmf_solve_batch_noalloc): its state
lives in the library's fixed per-device array.  Called through the C ABI,
it gives the flows, statuses and masks of pmf_solve_batch (bit for bit, and
those equal the oracle's) on two calls in a row on one handle, the second
with a smaller batch; a batch larger than the array is refused with
PMF_ELIMIT before any launch."""

import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_06004_amd import workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solve(pmf, torch, handle, dev, noalloc):
    total = sum(d.L for d in dev)
    flows = torch.full((total,), -7, dtype=torch.int64, device="cuda")
    status = torch.full((len(dev),), -7, dtype=torch.int32, device="cuda")
    fn = pmf.pmf_solve_batch_noalloc if noalloc else pmf.pmf_solve_batch
    rc = fn(handle, [d.c_struct() for d in dev], int(flows.data_ptr()), int(status.data_ptr()))
    torch.cuda.synchronize()
    masks = []
    for i, d in enumerate(dev):
        per = []
        for k in range(d.L):
            m = torch.empty((d.H, d.W), dtype=torch.uint8, device="cuda")
            assert pmf.pmf_extract_cut(handle, i, k, int(m.data_ptr())) == pmf.PMF_OK
            per.append(m.cpu().numpy().astype(bool))
        masks.append(np.stack(per))
    torch.cuda.synchronize()
    return rc, flows.cpu().numpy(), status.cpu().numpy(), masks


def test_noalloc_matches_solve_batch():
    import torch
    from paper_1509_06004_amd import pmf
    rng = np.random.default_rng(2024)
    big = [W.tiny_random(rng, 150, 110, 4, cmax=300, L=4, p_seed=0.02, lam_max=120),
           W.tiny_random(rng, 97, 131, 8, cmax=300, L=3, p_seed=0.02, lam_max=120),
           W.tiny_random(rng, 33, 70, 4, cmax=40, L=2, p_seed=0.1, lam_max=60)]
    small = [W.tiny_random(rng, 61, 45, 8, cmax=200, L=2, p_seed=0.05, lam_max=80)]
    say("no-alloc: first call", [(i.W, i.H, i.K, i.L) for i in big], "second", [(i.W, i.H, i.K, i.L) for i in small])
    h_ref = pmf.pmf_create(pmf.pmf_default_options(), int(torch.cuda.current_stream().cuda_stream))
    h = pmf.pmf_create(pmf.pmf_default_options(), int(torch.cuda.current_stream().cuda_stream))
    try:
        for insts in (big, small):
            dev = pmf.to_device(insts)
            rc0, f0, s0, m0 = _solve(pmf, torch, h_ref, dev, noalloc=False)
            rc1, f1, s1, m1 = _solve(pmf, torch, h, dev, noalloc=True)
            assert rc0 == pmf.PMF_OK and rc1 == pmf.PMF_OK, (rc0, rc1)
            assert (s0 == 0).all() and (s1 == s0).all(), (s0, s1)
            assert (f1 == f0).all(), (f0, f1)
            for a, b in zip(m0, m1):
                assert (a == b).all()
            o = 0
            for i, inst in enumerate(insts):
                for k in range(inst.L):
                    f, m = O.fifo_pr(inst, int(inst.lambdas[k]))
                    assert int(f1[o + k]) == f and (m1[i][k] == m).all(), (i, k)
                o += inst.L
            say("no-alloc call matches pmf_solve_batch and the oracle:", len(insts), "instances")
        # larger than the fixed array: refused before any launch
        huge = [W.tiny_random(rng, 640, 480, 8, cmax=10, L=30, p_seed=0.01, lam_max=50) for _ in range(4)]
        dev = pmf.to_device(huge)
        flows = torch.empty(sum(d.L for d in dev), dtype=torch.int64, device="cuda")
        rc = pmf.pmf_solve_batch_noalloc(h, [d.c_struct() for d in dev], int(flows.data_ptr()), 0)
        assert rc == pmf.PMF_ELIMIT, rc
    finally:
        pmf.pmf_destroy(h)
        pmf.pmf_destroy(h_ref)
