"""Python binding of libpmf (C ABI in ``include/pmf.h``): argument marshalling only.

Every step of the solve runs in the HIP library; PyTorch provides device
memory and the stream.  The library must be built (``python -m
paper_1509_06004_amd.build``); importing this module fails loudly otherwise.

Functions with the C names (``pmf_create``, ``pmf_solve_batch``,
``pmf_extract_cut``, ``pmf_destroy``, ...) wrap the ABI one to one;
:class:`Solver` is a small convenience layer over them.
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch  # loads the HIP runtime that libpmf then shares

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmf.so")

PMF_OK, PMF_EINVAL, PMF_EOVERFLOW, PMF_ENOMEM, PMF_EDEVICE = 0, 1, 2, 3, 4
PMF_ETIMEOUT, PMF_ENOTSOLVED, PMF_ERANGE, PMF_EBUSY, PMF_ELIMIT = 5, 6, 7, 8, 9
PMF_NOALLOC_BYTES = 64 << 20
INF = 1 << 30


class PmfError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__("%s: %s (code %d)" % (where, pmf_strerror(code), code))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("tile_w", ctypes.c_int32),
        ("tile_h", ctypes.c_int32),
        ("inner_iters", ctypes.c_int32),
        ("sweeps_per_relabel", ctypes.c_int32),
        ("local_bfs_iters", ctypes.c_int32),
        ("steps_per_sync", ctypes.c_int32),
        ("max_supersteps", ctypes.c_int64),
        ("use_graph", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("mem_budget", ctypes.c_int64),
        ("max_slots", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("lambda_chunk", ctypes.c_int32),
        ("exchange_rounds", ctypes.c_int32),
        ("tail_tiles", ctypes.c_int32),
        ("tail_inner_iters", ctypes.c_int32),
        ("tail_exchange_rounds", ctypes.c_int32),
        ("relabel_passes", ctypes.c_int32),
        ("orientation", ctypes.c_int32),
        ("gap", ctypes.c_int32),
        ("persist_tiles", ctypes.c_int32),
        ("persist_wgs", ctypes.c_int32),
        ("tail_sweep_exchanges", ctypes.c_int32),
    ]


class InstanceC(ctypes.Structure):
    _fields_ = [
        ("W", ctypes.c_int32),
        ("H", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("nlink", ctypes.c_void_p),
        ("cap_src", ctypes.c_void_p),
        ("cap_snk0", ctypes.c_void_p),
        ("snk_slope", ctypes.c_void_p),
        ("seed", ctypes.c_void_p),
        ("lambdas", ctypes.c_void_p),
    ]


class SessionInfo(ctypes.Structure):
    _fields_ = [
        ("free_bytes", ctypes.c_int64),
        ("largest_free", ctypes.c_int64),
        ("free_slots", ctypes.c_int32),
        ("admitted", ctypes.c_int32),
        ("running", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("supersteps", ctypes.c_int64),
        ("sweep_visits", ctypes.c_int64),
        ("global_relabels", ctypes.c_int64),
        ("bfs_passes", ctypes.c_int64),
        ("host_syncs", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("device_ns", ctypes.c_int64),
        ("px_init", ctypes.c_int64),
        ("px_sweep", ctypes.c_int64),
        ("px_relabel", ctypes.c_int64),
        ("px_cut", ctypes.c_int64),
        ("work_ns", ctypes.c_int64),
        ("sweep_ns", ctypes.c_int64),
        ("pass_ns", ctypes.c_int64),
        ("control_ns", ctypes.c_int64),
        ("work_launches", ctypes.c_int64),
        ("px_orient", ctypes.c_int64),
        ("px_init_x", ctypes.c_int64),
        ("px_cut_x", ctypes.c_int64),
        ("gap_kills", ctypes.c_int64),
        ("persist_launches", ctypes.c_int64),
        ("persist_supersteps", ctypes.c_int64),
        ("persist_ns", ctypes.c_int64),
        ("kernel_px", ctypes.c_int64 * 16),
    ]


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libpmf.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpmf.so is not built: run `python -m paper_1509_06004_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    sig = {
        "pmf_default_options": (None, [ctypes.POINTER(Options)]),
        "pmf_create": (ctypes.c_int, [ctypes.POINTER(Options), P, P, ctypes.c_size_t,
                                      ctypes.POINTER(P)]),
        "pmf_solve_batch": (ctypes.c_int, [P, ctypes.POINTER(InstanceC), ctypes.c_int32, P, P]),
        "pmf_solve_batch_noalloc": (ctypes.c_int, [P, ctypes.POINTER(InstanceC), ctypes.c_int32, P, P]),
        "pmf_solve_batch_async": (ctypes.c_int, [P, ctypes.POINTER(InstanceC), ctypes.c_int32, P, P]),
        "pmf_wait": (ctypes.c_int, [P]),
        "pmf_query_done": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int32)]),
        "pmf_extract_cut": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, P]),
        "pmf_destroy": (ctypes.c_int, [P]),
        "pmf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "pmf_query_bytes": (ctypes.c_int, [ctypes.POINTER(InstanceC), ctypes.c_int32,
                                           ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]),
        "pmf_check_instances": (ctypes.c_int, [ctypes.POINTER(InstanceC), ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int32)]),
        "pmf_get_stats": (ctypes.c_int, [P, ctypes.POINTER(Stats)]),
        "pmf_slot_stats": (ctypes.c_int, [P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
        "pmf_get_trace": (ctypes.c_int64, [P, P, ctypes.c_int64]),
        "pmf_parametric": (ctypes.c_int, [P, ctypes.POINTER(InstanceC), ctypes.c_int32, ctypes.c_int32, P, P,
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), P]),
        "pmf_breakpoints": (ctypes.c_int, [P, ctypes.POINTER(InstanceC), ctypes.c_int32, ctypes.c_int32, P, P, P,
                                           P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), P]),
        "pmf_extract_levels": (ctypes.c_int, [P, ctypes.c_int32, P]),
        "pmf_session_open": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_size_t]),
        "pmf_session_submit": (ctypes.c_int, [P, ctypes.POINTER(InstanceC), ctypes.c_int32, P, P,
                                              ctypes.POINTER(ctypes.c_int32)]),
        "pmf_session_step": (ctypes.c_int, [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
        "pmf_session_release": (ctypes.c_int, [P, ctypes.c_int32]),
        "pmf_session_query": (ctypes.c_int, [P, ctypes.POINTER(SessionInfo)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# One-to-one wrappers of the C ABI.
# ---------------------------------------------------------------------------

def pmf_strerror(code: int) -> str:
    return load_library().pmf_strerror(int(code)).decode()


def pmf_default_options() -> Options:
    o = Options()
    load_library().pmf_default_options(ctypes.byref(o))
    return o


def pmf_create(options: Optional[Options] = None, stream: int = 0, workspace: int = 0,
               ws_bytes: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    rc = load_library().pmf_create(ctypes.byref(options) if options is not None else None,
                                   ctypes.c_void_p(stream), ctypes.c_void_p(workspace),
                                   ctypes.c_size_t(ws_bytes), ctypes.byref(h))
    if rc != PMF_OK:
        raise PmfError(rc, "pmf_create")
    return h


def pmf_solve_batch(handle, instances: Sequence[InstanceC], flows_ptr: int, status_ptr: int) -> int:
    arr = (InstanceC * len(instances))(*instances)
    return load_library().pmf_solve_batch(handle, arr, len(instances), ctypes.c_void_p(flows_ptr),
                                          ctypes.c_void_p(status_ptr))


def pmf_solve_batch_noalloc(handle, instances: Sequence[InstanceC], flows_ptr: int, status_ptr: int) -> int:
    arr = (InstanceC * len(instances))(*instances)
    return load_library().pmf_solve_batch_noalloc(handle, arr, len(instances), ctypes.c_void_p(flows_ptr),
                                                  ctypes.c_void_p(status_ptr))


def pmf_solve_batch_async(handle, instances: Sequence[InstanceC], flows_ptr: int, status_ptr: int) -> int:
    arr = (InstanceC * len(instances))(*instances)
    return load_library().pmf_solve_batch_async(handle, arr, len(instances), ctypes.c_void_p(flows_ptr),
                                                ctypes.c_void_p(status_ptr))


def pmf_wait(handle) -> int:
    return load_library().pmf_wait(handle)


def pmf_query_done(handle) -> bool:
    done = ctypes.c_int32(0)
    rc = load_library().pmf_query_done(handle, ctypes.byref(done))
    if rc != PMF_OK:
        raise PmfError(rc, "pmf_query_done")
    return bool(done.value)


def pmf_extract_cut(handle, inst: int, lambda_idx: int, mask_ptr: int) -> int:
    return load_library().pmf_extract_cut(handle, int(inst), int(lambda_idx), ctypes.c_void_p(mask_ptr))


def pmf_extract_levels(handle, inst: int, levels_ptr: int) -> int:
    return load_library().pmf_extract_levels(handle, int(inst), ctypes.c_void_p(levels_ptr))


def pmf_destroy(handle) -> int:
    return load_library().pmf_destroy(handle)


def pmf_query_bytes(instances: Sequence[InstanceC], options: Optional[Options] = None) -> int:
    arr = (InstanceC * len(instances))(*instances)
    out = ctypes.c_size_t(0)
    rc = load_library().pmf_query_bytes(arr, len(instances),
                                        ctypes.byref(options) if options is not None else None,
                                        ctypes.byref(out))
    if rc != PMF_OK:
        raise PmfError(rc, "pmf_query_bytes")
    return int(out.value)


def pmf_check_instances(instances: Sequence[InstanceC]) -> Tuple[int, int]:
    arr = (InstanceC * len(instances))(*instances)
    bad = ctypes.c_int32(-1)
    rc = load_library().pmf_check_instances(arr, len(instances), ctypes.byref(bad))
    return rc, int(bad.value)


def pmf_slot_stats(handle, max_slots: int = 1 << 16) -> np.ndarray:
    """int64 [slots, 8]: finished, supersteps, sweeps, relabels, passes, lambdas
    done, pixels swept, pixels relaxed."""
    out = np.zeros((max_slots, 8), dtype=np.int64)
    n = ctypes.c_int32(0)
    rc = load_library().pmf_slot_stats(handle, out.ctypes.data, max_slots, ctypes.byref(n))
    if rc != PMF_OK:
        raise PmfError(rc, "pmf_slot_stats")
    return out[:min(n.value, max_slots)]


PMF_TRACE_COLS = 8
TRACE_FIELDS = ("sweep_tiles4", "sweep_tiles8", "pass_tiles4", "pass_tiles8", "sweep_ns", "pass_ns",
                "control_ns", "work_ns")


def pmf_parametric(handle, inst: "DeviceInstance", lam_lo: int, lam_hi: int, max_bp: int = 4096,
                   exit_map: bool = True):
    """All breakpoints of one instance over [lam_lo, lam_hi] (see the C
    declaration).  Returns (change points int32 array, F at lam_lo and at each
    change point int64 array, per-pixel exit lambda (int32 H x W device tensor,
    or None))."""
    bp = np.zeros(max(max_bp, 1), dtype=np.int32)
    fo = np.zeros(max(max_bp, 1) + 1, dtype=np.int64)
    nbp = ctypes.c_int32(0)
    ex = torch.empty((inst.H, inst.W), dtype=torch.int32, device=inst.cap_src.device) if exit_map else None
    c = inst.c_struct()
    rc = load_library().pmf_parametric(handle, ctypes.byref(c), int(lam_lo), int(lam_hi), bp.ctypes.data,
                                       fo.ctypes.data, int(max_bp), ctypes.byref(nbp),
                                       int(ex.data_ptr()) if ex is not None else None)
    if rc != PMF_OK:
        raise PmfError(rc, "pmf_parametric")
    n = nbp.value
    return bp[:n].copy(), fo[:n + 1].copy(), ex


def pmf_breakpoints(handle, inst: "DeviceInstance", lam_lo: int, lam_hi: int, max_bp: int = 4096):
    """Every real breakpoint of one instance over [lam_lo, lam_hi] (see the C
    declaration).  Returns (numerators int64, denominators int64, piece
    intercepts int64 [n + 1], piece slopes int64 [n + 1], per-pixel exit piece
    (int32 H x W device tensor))."""
    m = max(max_bp, 1)
    num = np.zeros(m, dtype=np.int64)
    den = np.zeros(m, dtype=np.int64)
    pa = np.zeros(m + 1, dtype=np.int64)
    pw = np.zeros(m + 1, dtype=np.int64)
    nbp = ctypes.c_int32(0)
    ex = torch.empty((inst.H, inst.W), dtype=torch.int32, device=inst.cap_src.device)
    c = inst.c_struct()
    rc = load_library().pmf_breakpoints(handle, ctypes.byref(c), int(lam_lo), int(lam_hi), num.ctypes.data,
                                        den.ctypes.data, pa.ctypes.data, pw.ctypes.data, int(max_bp),
                                        ctypes.byref(nbp), int(ex.data_ptr()))
    if rc != PMF_OK:
        raise PmfError(rc, "pmf_breakpoints")
    n = nbp.value
    return num[:n].copy(), den[:n].copy(), pa[:n + 1].copy(), pw[:n + 1].copy(), ex


def pmf_get_trace(handle) -> np.ndarray:
    """int64 [supersteps, 8] trace of the last solve run in timing mode (columns
    TRACE_FIELDS); empty without timing mode."""
    lib = load_library()
    rows = lib.pmf_get_trace(handle, None, 0)
    if rows < 0:
        raise PmfError(int(-rows), "pmf_get_trace")
    out = np.zeros((rows, PMF_TRACE_COLS), dtype=np.int64)
    if rows:
        got = lib.pmf_get_trace(handle, out.ctypes.data, rows)
        if got != rows:
            raise PmfError(PMF_EDEVICE, "pmf_get_trace")
    return out


def pmf_get_stats(handle) -> Dict[str, int]:
    s = Stats()
    rc = load_library().pmf_get_stats(handle, ctypes.byref(s))
    if rc != PMF_OK:
        raise PmfError(rc, "pmf_get_stats")
    out = {}
    for f, _ in Stats._fields_:
        v = getattr(s, f)
        out[f] = [int(x) for x in v] if f == "kernel_px" else int(v)
    return out


def pmf_session_open(handle, max_slots: int, pool_bytes: int = 0) -> int:
    return load_library().pmf_session_open(handle, int(max_slots), ctypes.c_size_t(pool_bytes))


def pmf_session_submit(handle, instances: Sequence[InstanceC], flows_ptr: int, status_ptr: int):
    """Returns (code, ids)."""
    arr = (InstanceC * len(instances))(*instances)
    ids = (ctypes.c_int32 * max(len(instances), 1))()
    rc = load_library().pmf_session_submit(handle, arr, len(instances), ctypes.c_void_p(flows_ptr),
                                           ctypes.c_void_p(status_ptr), ids)
    return rc, [int(ids[i]) for i in range(len(instances))] if rc == PMF_OK else []


def pmf_session_step(handle, supersteps: int, max_ids: int = 4096):
    """Returns (code, finished ids)."""
    buf = (ctypes.c_int32 * max_ids)()
    n = ctypes.c_int32(0)
    rc = load_library().pmf_session_step(handle, int(supersteps), buf, max_ids, ctypes.byref(n))
    return rc, [int(buf[i]) for i in range(min(n.value, max_ids))]


def pmf_session_release(handle, ident: int) -> int:
    return load_library().pmf_session_release(handle, int(ident))


def pmf_session_query(handle) -> Dict[str, int]:
    info = SessionInfo()
    rc = load_library().pmf_session_query(handle, ctypes.byref(info))
    if rc != PMF_OK:
        raise PmfError(rc, "pmf_session_query")
    return {f: int(getattr(info, f)) for f, _ in SessionInfo._fields_ if f != "reserved"}


# ---------------------------------------------------------------------------
# Device-resident instances (torch tensors) and a convenience solver.
# ---------------------------------------------------------------------------

class DeviceInstance:
    """Device copies of one instance's arrays; keeps the tensors alive."""

    def __init__(self, W, H, K, nlink, cap_src, cap_snk0, snk_slope, seed, lambdas):
        self.W, self.H, self.K = int(W), int(H), int(K)
        self.nlink, self.cap_src, self.cap_snk0 = nlink, cap_src, cap_snk0
        self.snk_slope, self.seed, self.lambdas = snk_slope, seed, lambdas
        self.L = int(lambdas.numel())

    def c_struct(self) -> InstanceC:
        def ptr(t):
            return 0 if t is None else int(t.data_ptr())
        return InstanceC(self.W, self.H, self.K, self.L, ptr(self.nlink), ptr(self.cap_src),
                         ptr(self.cap_snk0), ptr(self.snk_slope), ptr(self.seed), ptr(self.lambdas))


def to_device(insts, device="cuda", share: Optional[Dict[int, tuple]] = None,
              non_blocking: bool = False) -> List[DeviceInstance]:
    """Upload host instances (objects with the fields of ``workload.Instance``).
    Arrays that are the same numpy object (n-links of one image, shared
    constant planes) get one device copy.  A ``share`` dict passed in carries
    that over calls: it holds each uploaded array with its copy (keeping the
    array alive, so that a later object can never be taken for it)."""
    share = {} if share is None else share

    def up(a, dt):
        key = id(a)
        hit = share.get(key)
        if hit is None or hit[0] is not a:
            c = np.ascontiguousarray(a, dtype=dt)
            h = torch.from_numpy(c if c.flags.writeable else c.copy())
            if non_blocking:
                h = h.pin_memory()
            hit = (a, h.to(device, non_blocking=non_blocking))
            share[key] = hit
        return hit[1]

    out = []
    for inst in insts:
        out.append(DeviceInstance(inst.W, inst.H, inst.K, up(inst.nlink, np.int32), up(inst.cap_src, np.int32),
                                  up(inst.cap_snk0, np.int32), up(inst.snk_slope, np.int32),
                                  up(inst.seed, np.uint8), up(inst.lambdas, np.int32)))
    return out


class Solver:
    """Owns a pmf handle bound to a torch stream."""

    def __init__(self, options: Optional[Options] = None, stream: Optional[torch.cuda.Stream] = None,
                 workspace: Optional[torch.Tensor] = None, **overrides):
        if options is None:
            options = pmf_default_options()
        for k, v in overrides.items():
            setattr(options, k, v)
        self.options = options
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.workspace = workspace
        ws_ptr = int(workspace.data_ptr()) if workspace is not None else 0
        ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
        self.handle = pmf_create(options, int(self.stream.cuda_stream), ws_ptr, ws_bytes)
        self.last = []

    def solve(self, dev_insts: Sequence[DeviceInstance]) -> Tuple[torch.Tensor, torch.Tensor]:
        """Returns (flows int64 [sum L], status int32 [n]) on the device."""
        total = sum(d.L for d in dev_insts)
        dev = dev_insts[0].lambdas.device if dev_insts else torch.device("cuda")
        flows = torch.empty(total, dtype=torch.int64, device=dev)
        status = torch.empty(len(dev_insts), dtype=torch.int32, device=dev)
        rc = pmf_solve_batch(self.handle, [d.c_struct() for d in dev_insts], int(flows.data_ptr()),
                             int(status.data_ptr()))
        if rc != PMF_OK:
            raise PmfError(rc, "pmf_solve_batch")
        self.last = list(dev_insts)
        return flows, status

    def solve_async(self, dev_insts: Sequence[DeviceInstance]) -> Tuple[torch.Tensor, torch.Tensor]:
        """Start a solve and return at once; the tensors are complete after wait()."""
        total = sum(d.L for d in dev_insts)
        dev = dev_insts[0].lambdas.device if dev_insts else torch.device("cuda")
        flows = torch.empty(total, dtype=torch.int64, device=dev)
        status = torch.empty(len(dev_insts), dtype=torch.int32, device=dev)
        self._async_args = [d.c_struct() for d in dev_insts]
        rc = pmf_solve_batch_async(self.handle, self._async_args, int(flows.data_ptr()), int(status.data_ptr()))
        if rc != PMF_OK:
            raise PmfError(rc, "pmf_solve_batch_async")
        self.last = list(dev_insts)
        return flows, status

    def wait(self) -> None:
        rc = pmf_wait(self.handle)
        if rc != PMF_OK:
            raise PmfError(rc, "pmf_solve_batch_async")

    def done(self) -> bool:
        return pmf_query_done(self.handle)

    def extract_cut(self, inst: int, lambda_idx: int) -> torch.Tensor:
        d = self.last[inst]
        out = torch.empty((d.H, d.W), dtype=torch.uint8, device=d.lambdas.device)
        rc = pmf_extract_cut(self.handle, inst, lambda_idx, int(out.data_ptr()))
        if rc != PMF_OK:
            raise PmfError(rc, "pmf_extract_cut")
        return out

    def stats(self) -> Dict[str, int]:
        return pmf_get_stats(self.handle)

    def close(self):
        if self.handle is not None:
            pmf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
