"""Continuous-batching serving loop over one resident libpmf session.

Requests (one image with several seeds, each with its own lambda schedule)
arrive at scheduled times.  The server keeps a FIFO of arrived requests and
admits them, whole, while the backend has free instance slots and pool memory
(admission by free memory) and the work in flight stays under a bound.
Admitted requests join the running launches at the next superstep, so work of
different requests overlaps on the device; a request completes when all its
instances have finished, and its results (flow values and one nested-level
byte per pixel per seed) are then copied to the host.  Latency is measured from
the scheduled arrival to the results being on the host.

The scheduling mirrors the paper's dynamic scheduler (Sec. 3.3.1): work goes to
free capacity in FIFO order as soon as capacity frees up, instead of a fixed
static assignment; here the capacity is device slots and memory of one GPU.

Backends share one interface, so the server logic is tested on the CPU with a
fake backend and run on the GPU with :class:`PmfBackend`.
"""

from __future__ import annotations

import dataclasses
import itertools
import time
from collections import deque
from typing import Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Result:
    flows: np.ndarray   # int64 [L] per instance
    levels: np.ndarray  # uint8 [H, W]: mask of lambda k is levels > k
    status: int


@dataclasses.dataclass
class RequestRecord:
    index: int
    arrival: float
    n_inst: int
    solves: int
    admitted: float = float("nan")
    finished: float = float("nan")
    failed: Optional[str] = None
    results: Optional[List[Result]] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Backend:
    """Interface of a solver backend (all times host wall-clock)."""

    def bytes_needed(self, insts) -> int:
        raise NotImplementedError

    def free_bytes(self) -> int:
        raise NotImplementedError

    def capacity(self) -> int:
        """Bytes of the whole pool: a request needing more can never run."""
        raise NotImplementedError

    def stage(self, insts):
        """Start moving a request's inputs to the device (returns a token for
        `ready` and `submit`; None when the backend has nothing to stage)."""
        return None

    def ready(self, staged) -> bool:
        """Whether the staged inputs have arrived (never blocks)."""
        return True

    def submit(self, insts, staged=None) -> Optional[List[int]]:
        """Admit all instances (ids) or none (None)."""
        raise NotImplementedError

    def step(self) -> List[int]:
        """Advance the device; ids of instances that finished."""
        raise NotImplementedError

    def fetch(self, ids: Sequence[int]) -> List[Result]:
        raise NotImplementedError

    def release(self, ids: Sequence[int]) -> None:
        raise NotImplementedError

    def reset(self) -> None:
        """Drop every admitted instance and free all slots and memory."""
        raise NotImplementedError


class PmfBackend(Backend):
    """libpmf session on one GPU (inputs uploaded per request)."""

    def __init__(self, max_slots: int = 4096, pool_bytes: int = 0, supersteps: int = 16, lambda_chunk: int = 0,
                 **options):
        import torch
        from . import pmf
        self.torch, self.pmf = torch, pmf
        opts = pmf.pmf_default_options()
        for k, v in options.items():
            setattr(opts, k, v)
        self.stream = torch.cuda.current_stream()
        self.copy_stream = torch.cuda.Stream()
        self.handle = pmf.pmf_create(opts, int(self.stream.cuda_stream))
        rc = pmf.pmf_session_open(self.handle, max_slots, pool_bytes)
        if rc != pmf.PMF_OK:
            raise pmf.PmfError(rc, "pmf_session_open")
        self.options = opts
        self.max_slots, self.pool_arg = max_slots, pool_bytes
        self.owner_of: Dict[int, int] = {}
        self.pending: Dict[int, int] = {}
        self.supersteps = supersteps
        # every request instance is split into chunks of lambda_chunk lambdas
        # (0: not split), each a device instance of its own: more parallel
        # work per request, but each chunk starts cold.  A stream of requests
        # brings parallel work of its own, so whole warm chains serve more.
        self.chunk = int(lambda_chunk) if int(lambda_chunk) > 0 else 1 << 30
        self.groups: Dict[int, List[int]] = {}  # first device id -> device ids of one instance
        self.pool_bytes = pmf.pmf_session_query(self.handle)["free_bytes"]
        self.live: Dict[int, tuple] = {}  # id -> (device inputs, flows view, status view, L, H, W)

    def _chunks(self, inst):
        L = int(inst.lambdas.shape[0])
        return [(a, min(L, a + self.chunk)) for a in range(0, L, self.chunk)]

    def bytes_needed(self, insts) -> int:
        fake = []
        for i in insts:
            for a, b in self._chunks(i):
                fake.append(self.pmf.InstanceC(i.W, i.H, i.K, b - a, 1, 1, 1, 0, 0, 1))
        return self.pmf.pmf_query_bytes(fake, self.options)

    def free_bytes(self) -> int:
        return self.pmf.pmf_session_query(self.handle)["largest_free"]

    def capacity(self) -> int:
        return self.pool_bytes

    def stage(self, insts):
        """Upload the request's inputs from pinned host memory on a copy stream
        of their own, so that the transfer overlaps with the supersteps that
        are running; the session's stream waits for it before the request's
        first launch (by then it has long finished)."""
        torch, pmf = self.torch, self.pmf
        with torch.cuda.stream(self.copy_stream):
            dev = pmf.to_device(insts, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        for d in dev:  # the tensors are used on the session's stream from now on
            for t in (d.nlink, d.cap_src, d.cap_snk0, d.snk_slope, d.seed, d.lambdas):
                t.record_stream(self.stream)
        return dev, ev

    def ready(self, staged) -> bool:
        return staged is None or staged[1].query()

    def submit(self, insts, staged=None) -> Optional[List[int]]:
        """One id per request instance (the id of its first chunk)."""
        torch, pmf = self.torch, self.pmf
        if staged is not None:
            dev, ev = staged
            self.stream.wait_event(ev)
        else:
            dev = pmf.to_device(insts)
        subs, owner = [], []
        for j, d in enumerate(dev):
            for a, b in self._chunks(insts[j]):
                subs.append(pmf.DeviceInstance(d.W, d.H, d.K, d.nlink, d.cap_src, d.cap_snk0, d.snk_slope,
                                               d.seed, d.lambdas[a:b]))
                owner.append(j)
        total = sum(d.L for d in subs)
        flows = torch.empty(total, dtype=torch.int64, device="cuda")
        status = torch.empty(len(subs), dtype=torch.int32, device="cuda")
        rc, ids = pmf.pmf_session_submit(self.handle, [d.c_struct() for d in subs], int(flows.data_ptr()),
                                         int(status.data_ptr()))
        if rc == pmf.PMF_EBUSY:
            return None
        if rc != pmf.PMF_OK:
            raise pmf.PmfError(rc, "pmf_session_submit")
        firsts, off, pos = [], 0, 0
        for j, d in enumerate(dev):
            n_ch = len(self._chunks(insts[j]))
            grp = ids[pos:pos + n_ch]
            self.groups[grp[0]] = grp
            self.live[grp[0]] = (d, flows[off:off + d.L], status[pos:pos + n_ch], d.L, d.H, d.W,
                                 (flows, status, subs))
            firsts.append(grp[0])
            off += d.L
            pos += n_ch
        for f in firsts:
            for i in self.groups[f]:
                self.owner_of[i] = f
        for f in firsts:
            self.pending[f] = len(self.groups[f])
        return firsts

    def step(self) -> List[int]:
        rc, done = self.pmf.pmf_session_step(self.handle, self.supersteps)
        if rc != self.pmf.PMF_OK:
            raise self.pmf.PmfError(rc, "pmf_session_step")
        out = []
        for i in done:
            f = self.owner_of.get(i)
            if f is None:
                continue
            self.pending[f] -= 1
            if self.pending[f] == 0:
                out.append(f)
        return out

    def fetch(self, ids: Sequence[int]) -> List[Result]:
        torch, pmf = self.torch, self.pmf
        lv, fl, stv = [], [], []
        for f in ids:
            d, flows, status, L, H, W, _ = self.live[f]
            out = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
            tmp = torch.empty((H, W), dtype=torch.uint8, device="cuda")
            for i in self.groups[f]:
                rc = pmf.pmf_extract_levels(self.handle, i, int(tmp.data_ptr()))
                if rc != pmf.PMF_OK:
                    raise pmf.PmfError(rc, "pmf_extract_levels")
                out += tmp  # chunks partition the schedule; the sets are nested
            lv.append(out)
            fl.append(flows)
            stv.append(status)
        flows_h = [f.to("cpu", non_blocking=True) for f in fl]
        levels_h = [x.to("cpu", non_blocking=True) for x in lv]
        status_h = [s.to("cpu", non_blocking=True) for s in stv]
        torch.cuda.current_stream().synchronize()
        res = []
        for f, l, s in zip(flows_h, levels_h, status_h):
            st = s.numpy()
            code = int(st[st != 0][0]) if (st != 0).any() else 0
            res.append(Result(f.numpy(), l.numpy(), code))
        return res

    def release(self, ids: Sequence[int]) -> None:
        for f in ids:
            for i in self.groups.pop(f):
                rc = self.pmf.pmf_session_release(self.handle, i)
                if rc != self.pmf.PMF_OK:
                    raise self.pmf.PmfError(rc, "pmf_session_release")
                self.owner_of.pop(i, None)
            self.pending.pop(f, None)
            self.live.pop(f, None)

    def reset(self) -> None:
        rc = self.pmf.pmf_session_open(self.handle, self.max_slots, self.pool_arg)
        if rc != self.pmf.PMF_OK:
            raise self.pmf.PmfError(rc, "pmf_session_open")
        self.groups.clear()
        self.live.clear()
        self.owner_of.clear()
        self.pending.clear()

    def stats(self) -> Dict[str, int]:
        return self.pmf.pmf_get_stats(self.handle)

    def close(self):
        if self.handle is not None:
            self.pmf.pmf_destroy(self.handle)
            self.handle = None


@dataclasses.dataclass
class ServeReport:
    qps: float
    offered: int
    completed: int
    failed: int
    duration_s: float
    solves: int
    solves_per_s: float
    p50_ms: float
    p99_ms: float
    censored: int
    max_queue: int
    records: List[RequestRecord]

    def summary(self) -> dict:
        return {"qps": self.qps, "offered_requests": self.offered, "completed_requests": self.completed,
                "failed_requests": self.failed, "duration_s": round(self.duration_s, 3),
                "solves": self.solves, "solves_per_s": round(self.solves_per_s, 2),
                "latency_ms": {"p50": round(self.p50_ms, 2), "p99": round(self.p99_ms, 2)},
                "unfinished_at_end": self.censored, "max_queue": self.max_queue}


class Server:
    """FIFO admission by free memory, continuous batching, latency accounting."""

    def __init__(self, backend: Backend, max_inflight_instances: int = 1 << 30, keep_results: bool = False,
                 clock=time.perf_counter, sleep=time.sleep, stage_ahead: int = 8):
        self.backend = backend
        self.stage_ahead = stage_ahead  # queued requests whose inputs are moved to the device ahead of admission
        self.max_inflight = max_inflight_instances
        self.keep_results = keep_results
        self.clock = clock
        self.sleep = sleep

    def run(self, arrivals: Sequence[float], make_request, duration_s: float, warmup_s: float = 0.0,
            qps: float = 0.0, drain: bool = False) -> ServeReport:
        """Serve requests arriving at `arrivals` (seconds from the start);
        `make_request(i)` returns the host instances of request i.  Requests
        arriving in [warmup_s, warmup_s + duration_s) are measured; the run
        stops at warmup_s + duration_s (or when everything is done, with
        `drain`)."""
        be = self.backend
        t0 = self.clock()
        end = warmup_s + duration_s
        pending: deque = deque()
        inflight: Dict[int, RequestRecord] = {}  # instance id -> record
        left: Dict[int, int] = {}                # record index -> unfinished instances
        ids_of: Dict[int, List[int]] = {}
        records: List[RequestRecord] = []
        nxt = 0
        n_inflight = 0
        max_queue = 0
        while True:
            now = self.clock() - t0
            while nxt < len(arrivals) and arrivals[nxt] <= now and arrivals[nxt] < end:
                insts = make_request(nxt)
                rec = RequestRecord(index=nxt, arrival=arrivals[nxt], n_inst=len(insts),
                                    solves=sum(i.L for i in insts))
                records.append(rec)
                pending.append([rec, insts, None])
                nxt += 1
            # inputs of the first queued requests start moving to the device
            # at once (bounded), overlapping with the work in flight
            for item in itertools.islice(pending, self.stage_ahead):
                if item[2] is None and item[0].failed is None:
                    try:
                        item[2] = ("staged", be.stage(item[1]))
                    except Exception as exc:  # a failed upload fails that request only
                        item[0].failed = repr(exc)
            max_queue = max(max_queue, len(pending))
            # admission: whole requests, FIFO, while memory, slots and the bound allow
            while pending and (n_inflight == 0 or n_inflight + pending[0][0].n_inst <= self.max_inflight):
                rec, insts, staged = pending[0]
                if rec.failed is not None:
                    pending.popleft()
                    rec.finished = self.clock() - t0
                    continue
                if be.bytes_needed(insts) > be.capacity():
                    pending.popleft()
                    rec.failed = "request larger than the whole pool"
                    rec.finished = self.clock() - t0
                    continue
                token = staged[1] if staged is not None else None
                if staged is not None and not be.ready(token):
                    break  # FIFO: wait for its upload
                try:
                    ids = be.submit(insts) if token is None else be.submit(insts, token)
                except Exception as exc:  # a failed request must not stop the others
                    pending.popleft()
                    rec.failed = repr(exc)
                    rec.finished = self.clock() - t0
                    continue
                if ids is None:
                    break
                pending.popleft()
                rec.admitted = self.clock() - t0
                ids_of[rec.index] = ids
                left[rec.index] = len(ids)
                for i in ids:
                    inflight[i] = rec
                n_inflight += len(ids)
            now = self.clock() - t0
            if now >= end and not drain:
                break
            if not inflight:
                if nxt >= len(arrivals) and not pending:
                    break
                if not pending and nxt < len(arrivals):
                    self.sleep(max(0.0, min(arrivals[nxt] - now, 0.002)))
                elif pending:
                    self.sleep(0.0002)  # the head request's inputs are still on their way
                continue
            try:
                done = be.step()
            except Exception as exc:
                # the device step failed: fail every request in flight and
                # hand its slots and memory back (if that fails too, the
                # backend starts afresh, which frees everything)
                failed = {rec.index: rec for rec in inflight.values()}
                for idx, rec in failed.items():
                    rec.failed = repr(exc)
                    rec.finished = self.clock() - t0
                    ids = ids_of.pop(idx, [])
                    try:
                        be.release(ids)
                    except Exception:
                        be.reset()
                inflight.clear()
                left.clear()
                n_inflight = 0
                continue
            finished_recs = []
            for i in done:
                rec = inflight.pop(i, None)
                if rec is None:
                    continue
                left[rec.index] -= 1
                if left[rec.index] == 0:
                    finished_recs.append(rec)
            for rec in finished_recs:
                ids = ids_of.pop(rec.index)
                res = be.fetch(ids)
                rec.finished = self.clock() - t0
                if self.keep_results:
                    rec.results = res
                be.release(ids)
                n_inflight -= len(ids)
                del left[rec.index]
        dur = self.clock() - t0
        window = [r for r in records if warmup_s <= r.arrival < end]
        ok = [r for r in window if r.failed is None and np.isfinite(r.finished)]
        # requests still unfinished at the end count with (end of run - arrival),
        # a lower bound of their latency, so that overload shows in p50/p99
        open_ = [r for r in window if r.failed is None and not np.isfinite(r.finished)]
        lat_list = [r.latency for r in ok] + [dur - r.arrival for r in open_]
        lat = np.array(lat_list) * 1e3 if lat_list else np.array([float("nan")])
        # throughput counts the solves of every request that finished inside
        # the measured time span, whenever it arrived (under overload the
        # span is spent on requests that queued before it)
        stop = min(dur, end) if not drain else dur
        measured_solves = sum(r.solves for r in records
                              if r.failed is None and np.isfinite(r.finished) and warmup_s <= r.finished <= stop)
        span = max(stop - warmup_s, 1e-9)
        return ServeReport(qps=qps, offered=len(window), completed=len(ok),
                           failed=sum(r.failed is not None for r in window), duration_s=dur,
                           solves=measured_solves, solves_per_s=measured_solves / span,
                           p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                           censored=len(open_), max_queue=max_queue, records=records)
