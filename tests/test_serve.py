"""Host-only tests of the serving loop: a fake backend (the CPU oracle behind
the backend interface, a byte budget in place of device memory) exercises
admission by free memory, FIFO order, continuous batching, latency accounting
and failure isolation without a GPU."""

from collections import deque

import numpy as np
import pytest

from oracle import oracle as O
from paper_1509_06004_amd import workload as W
from paper_1509_06004_amd.serve import Backend, Result, Server


class OracleBackend(Backend):
    def __init__(self, budget_bytes, per_step=1, bytes_per_px=64, fail_submit_at=None, fail_step_at=None):
        self.budget = budget_bytes
        self.per_step = per_step
        self.bpp = bytes_per_px
        self.used = 0
        self.max_used = 0
        self.next_id = 0
        self.queue = deque()
        self.live = {}
        self.submits = 0
        self.steps = 0
        self.fail_submit_at = fail_submit_at
        self.fail_step_at = fail_step_at
        self.admit_order = []

    def bytes_needed(self, insts):
        return sum(i.W * i.H * (self.bpp + i.L) for i in insts)

    def free_bytes(self):
        return self.budget - self.used

    def capacity(self):
        return self.budget

    def submit(self, insts):
        self.submits += 1
        if self.fail_submit_at is not None and self.submits == self.fail_submit_at:
            raise RuntimeError("injected submit failure")
        need = self.bytes_needed(insts)
        if need > self.free_bytes():
            return None
        ids = []
        for inst in insts:
            i = self.next_id
            self.next_id += 1
            self.live[i] = (inst, None)
            self.queue.append(i)
            ids.append(i)
        self.used += need
        self.max_used = max(self.max_used, self.used)
        self.admit_order.append(ids[0] if ids else None)
        return ids

    def step(self):
        self.steps += 1
        if self.fail_step_at is not None and self.steps == self.fail_step_at:
            raise RuntimeError("injected step failure")
        done = []
        for _ in range(min(self.per_step, len(self.queue))):
            i = self.queue.popleft()
            inst, _ = self.live[i]
            flows, masks = O.solve_chain(inst)
            self.live[i] = (inst, Result(flows, masks.sum(axis=0).astype(np.uint8), 0))
            done.append(i)
        return done

    def fetch(self, ids):
        return [self.live[i][1] for i in ids]

    def release(self, ids):
        for i in ids:
            inst, _ = self.live.pop(i)
            self.used -= self.bytes_needed([inst])
            if i in self.queue:
                self.queue.remove(i)

    def reset(self):
        self.live.clear()
        self.queue.clear()
        self.used = 0


def make_stream(n, seed=3):
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n):
        k = int(rng.integers(1, 4))
        reqs.append([W.tiny_random(rng, int(rng.integers(3, 9)), int(rng.integers(3, 9)),
                                   4 if r % 2 else 8, cmax=30, L=int(rng.integers(1, 4)), p_seed=0.1,
                                   lam_max=40) for _ in range(k)])
    arrivals = np.sort(rng.uniform(0, 0.05, size=n))
    return arrivals, reqs


def check_results(rec, insts):
    assert rec.results is not None and len(rec.results) == len(insts)
    for inst, res in zip(insts, rec.results):
        flows, masks = O.solve_chain(inst)
        assert (res.flows == flows).all()
        for k in range(inst.L):
            assert ((res.levels > k) == masks[k]).all()


def test_all_requests_complete_with_oracle_results():
    arrivals, reqs = make_stream(24)
    be = OracleBackend(budget_bytes=1 << 30, per_step=2)
    rep = Server(be, keep_results=True).run(arrivals, lambda i: reqs[i], duration_s=1.0, drain=True)
    assert rep.completed == 24 and rep.failed == 0 and rep.censored == 0
    for rec in rep.records:
        check_results(rec, reqs[rec.index])
        assert rec.finished >= rec.admitted >= rec.arrival
    assert rep.p50_ms <= rep.p99_ms
    assert rep.solves == sum(i.L for r in reqs for i in r)


def test_admission_respects_memory_and_fifo():
    arrivals, reqs = make_stream(30, seed=5)
    be0 = OracleBackend(budget_bytes=1)
    largest = max(be0.bytes_needed(r) for r in reqs)
    be = OracleBackend(budget_bytes=largest, per_step=1)  # room for about one request
    burst = np.zeros_like(arrivals)  # everything arrives at once
    rep = Server(be, keep_results=True).run(burst, lambda i: reqs[i], duration_s=1.0, drain=True)
    assert rep.completed == 30
    assert be.max_used <= largest
    assert rep.max_queue > 1  # requests had to wait for memory
    adm = [r.admitted for r in sorted(rep.records, key=lambda r: r.index)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))  # FIFO


def test_inflight_bound_limits_concurrency():
    arrivals, reqs = make_stream(12, seed=7)
    be = OracleBackend(budget_bytes=1 << 30, per_step=1)
    srv = Server(be, max_inflight_instances=2, keep_results=True)
    rep = srv.run(arrivals, lambda i: reqs[i], duration_s=1.0, drain=True)
    assert rep.completed == 12
    for rec in rep.records:
        check_results(rec, reqs[rec.index])


def test_failed_submit_isolated():
    arrivals, reqs = make_stream(10, seed=9)
    be = OracleBackend(budget_bytes=1 << 30, per_step=3, fail_submit_at=3)
    rep = Server(be, keep_results=True).run(arrivals, lambda i: reqs[i], duration_s=1.0, drain=True)
    assert rep.failed == 1 and rep.completed == 9
    bad = [r for r in rep.records if r.failed]
    assert len(bad) == 1 and "injected" in bad[0].failed


def test_failed_step_fails_only_inflight_requests():
    arrivals, reqs = make_stream(10, seed=11)
    be = OracleBackend(budget_bytes=1 << 30, per_step=1, fail_step_at=2)
    rep = Server(be).run(arrivals, lambda i: reqs[i], duration_s=1.0, drain=True)
    assert rep.failed >= 1 and rep.completed + rep.failed == 10
    # the failed requests' slots and memory went back to the backend
    assert be.used == 0 and not be.live and not be.queue


def test_failed_release_resets_backend():
    arrivals, reqs = make_stream(10, seed=12)

    class BadRelease(OracleBackend):
        resets = 0

        def release(self, ids):
            if self.steps == self.fail_step_at:
                raise RuntimeError("injected release failure")
            super().release(ids)

        def reset(self):
            self.resets += 1
            super().reset()

    be = BadRelease(budget_bytes=1 << 30, per_step=1, fail_step_at=2)
    rep = Server(be).run(arrivals, lambda i: reqs[i], duration_s=1.0, drain=True)
    assert be.resets >= 1 and rep.failed >= 1 and rep.completed + rep.failed == 10
    assert be.used == 0 and not be.live


def test_request_larger_than_pool_fails_fast():
    arrivals, reqs = make_stream(5, seed=13)
    be = OracleBackend(budget_bytes=1)
    rep = Server(be).run(arrivals, lambda i: reqs[i], duration_s=1.0, drain=True)
    assert rep.failed == 5 and rep.completed == 0


class SimClock:
    """Simulated time: advances only when the backend steps or the server sleeps."""

    def __init__(self):
        self.t = 0.0

    def clock(self):
        return self.t

    def sleep(self, d):
        self.t += max(d, 1e-4)


def test_overload_reports_censored_latency():
    """A backend too slow for the offered load: requests left unfinished at the
    end still count in the latency percentiles (as lower bounds)."""
    rng = np.random.default_rng(17)
    reqs = [[W.tiny_random(rng, 6, 6, 4, cmax=40, L=2, p_seed=0.05)] for _ in range(40)]
    arrivals = np.linspace(0.0, 0.05, 40)
    sim = SimClock()

    class Slow(OracleBackend):
        def step(self):
            sim.t += 0.01  # each step takes 10 ms of simulated time
            return super().step()

    be = Slow(budget_bytes=1 << 30, per_step=1)
    rep = Server(be, clock=sim.clock, sleep=sim.sleep).run(arrivals, lambda i: reqs[i], duration_s=0.06,
                                                          drain=False)
    assert rep.offered == 40
    assert rep.censored + rep.completed + rep.failed == 40
    assert rep.completed <= 7 and rep.censored >= 33
    assert np.isfinite(rep.p99_ms) and rep.p99_ms >= rep.p50_ms
    # every unfinished request counts at least (end - arrival)
    assert rep.p50_ms >= 0.0


def test_overload_throughput_counts_backlog_finished_in_window():
    """Throughput counts every request that finishes inside the measured span,
    also those that queued during the warmup; latency counts the requests that
    arrived inside it."""
    rng = np.random.default_rng(18)
    reqs = [[W.tiny_random(rng, 5, 5, 4, cmax=30, L=2, p_seed=0.05)] for _ in range(30)]
    arrivals = np.linspace(0.0, 0.05, 30)  # all arrive before the measured span ends
    sim = SimClock()

    class Slow(OracleBackend):
        def step(self):
            sim.t += 0.01
            return super().step()

    be = Slow(budget_bytes=1 << 30, per_step=1)
    rep = Server(be, clock=sim.clock, sleep=sim.sleep).run(arrivals, lambda i: reqs[i], duration_s=0.1,
                                                          warmup_s=0.03, drain=False)
    # requests arriving in [0.03, 0.13): those at or after 0.03
    assert rep.offered == int((arrivals >= 0.03).sum())
    # every solve counted belongs to a request that finished inside the span,
    # and requests from the warmup backlog are among them
    assert rep.solves > 0 and rep.solves % 2 == 0
    assert rep.solves > 2 * rep.completed


class StagingBackend(OracleBackend):
    """Uploads take a number of polls to arrive: admission must wait for them
    without blocking, in FIFO order, and requests still come out exact."""

    def __init__(self, *a, polls=3, **k):
        super().__init__(*a, **k)
        self.polls = polls
        self.staged = 0
        self.not_ready = 0

    def stage(self, insts):
        self.staged += 1
        return {"left": self.polls, "insts": insts}

    def ready(self, token):
        token["left"] -= 1
        if token["left"] > 0:
            self.not_ready += 1
            return False
        return True

    def submit(self, insts, staged=None):
        assert staged is not None and staged["left"] <= 0 and staged["insts"] is insts
        return super().submit(insts)


def test_staged_uploads_gate_admission_in_order():
    rng = np.random.default_rng(77)
    reqs = [[W.tiny_random(rng, 5, 4, 4, cmax=9, L=2, p_seed=0.1, lam_max=20)] for _ in range(6)]
    be = StagingBackend(1 << 30, per_step=1, polls=3)
    sim = SimClock()
    srv = Server(be, keep_results=True, clock=sim.clock, sleep=sim.sleep, stage_ahead=2)
    rep = srv.run([0.0] * len(reqs), lambda i: reqs[i], duration_s=100.0, drain=True)
    assert rep.completed == len(reqs) and be.staged == len(reqs) and be.not_ready > 0
    assert be.admit_order == sorted(be.admit_order)
    for rec in rep.records:
        inst = reqs[rec.index][0]
        flows, _ = O.solve_chain(inst)
        assert list(rec.results[0].flows) == list(flows)
