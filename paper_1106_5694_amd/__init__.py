"""Deep Greedy Switching (DGS) for the Linear Sum Assignment Problem on
AMD Instinct MI355X (gfx950).

Python binding of ``libdgs.so`` (C ABI in ``include/dgs.h``).  This module
only marshals arguments: every step of the solver runs in the library's
HIP kernels.  There is no CPU fallback -- if the library is missing or no
GPU is present, calls raise.

Inputs are either host arrays (numpy, or CPU torch tensors) or ROCm torch
tensors on the device (then the library reads and writes device memory in
place, on torch's current stream).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgs.so")

DGS_OK, DGS_E_INVAL, DGS_E_RANGE, DGS_E_NOMEM, DGS_E_DEVICE, DGS_E_AGAIN = range(6)
DGS_DEVICE_PTRS = 0x1
DGS_PROFILE = 0x2
DGS_AUTOTUNE = 0x4
DGS_PARALLEL = 0x8
DGS_LAZY = 0x10
DGS_GLOBAL_GREEDY = 0x20
PHASES = ("range", "init", "layout", "scan", "switch")
MAX_ABS_BENEFIT = (1 << 29) - 1

# Every symbol include/dgs.h declares.
EXPORTS = (
    "dgs_solve", "dgs_solve_ex", "dgs_solve_rect", "dgs_solve_batched", "dgs_diff_eval",
    "dgs_server_footprint", "dgs_server_create", "dgs_server_submit", "dgs_server_poll",
    "dgs_server_wait", "dgs_server_stats_get", "dgs_server_destroy",
    "dgs_status_string", "dgs_last_error", "dgs_version", "dgs_release_cached",
    "dgs_batch_plan_create", "dgs_batch_plan_benefit", "dgs_batch_plan_assign", "dgs_batch_plan_run",
    "dgs_batch_plan_config", "dgs_batch_plan_destroy", "dgs_solve_noalloc",
)
NOALLOC_MAX_N = 4096


class DGSError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("max_switches", ctypes.c_int64),
                ("init_assign", ctypes.c_void_p),
                ("flags", ctypes.c_uint32),
                ("stream", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("initial_benefit", ctypes.c_int64),
                ("total_benefit", ctypes.c_int64),
                ("switches", ctypes.c_int64),
                ("rescans", ctypes.c_int64),
                ("stalls", ctypes.c_int64),
                ("device_ms", ctypes.c_float),
                ("phase_ms", ctypes.c_float * 5),
                ("rounds", ctypes.c_int64),
                ("attempts", ctypes.c_int64)]

    def as_dict(self):
        return dict(initial_benefit=int(self.initial_benefit), total_benefit=int(self.total_benefit),
                    switches=int(self.switches), rescans=int(self.rescans), stalls=int(self.stalls),
                    rounds=int(self.rounds), attempts=int(self.attempts), device_ms=float(self.device_ms),
                    phase_ms={p: float(self.phase_ms[i]) for i, p in enumerate(PHASES)})


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64),
                ("max_slots", ctypes.c_int32),
                ("max_n", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("resident", ctypes.c_int64),
                ("inst_per_s", ctypes.c_double), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libdgs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1106_5694_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    L.dgs_solve.argtypes = [P, i32, P]
    L.dgs_solve_ex.argtypes = [P, i32, P, ctypes.POINTER(Options), ctypes.POINTER(Result)]
    L.dgs_solve_rect.argtypes = [P, i32, i32, P, ctypes.POINTER(Options), ctypes.POINTER(Result)]
    L.dgs_solve_noalloc.argtypes = [P, i32, P, ctypes.POINTER(Options), ctypes.POINTER(Result)]
    L.dgs_solve_batched.argtypes = [i32, P, P, P, P, ctypes.POINTER(Options)]
    L.dgs_diff_eval.argtypes = [P, i32, P, P, P, ctypes.POINTER(Options), ctypes.POINTER(Result)]
    L.dgs_server_footprint.argtypes = [i32]
    L.dgs_server_footprint.restype = ctypes.c_uint64
    L.dgs_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(P)]
    L.dgs_server_submit.argtypes = [P, P, i32, ctypes.POINTER(ctypes.c_uint64)]
    L.dgs_server_poll.argtypes = [P, ctypes.c_uint64, P, ctypes.POINTER(Result)]
    L.dgs_server_wait.argtypes = [P, ctypes.c_uint64, P, ctypes.POINTER(Result), ctypes.c_int64]
    L.dgs_server_stats_get.argtypes = [P, ctypes.POINTER(ServerStats)]
    L.dgs_server_destroy.argtypes = [P]
    L.dgs_server_destroy.restype = None
    L.dgs_batch_plan_create.argtypes = [i32, P, ctypes.POINTER(Options), ctypes.POINTER(P)]
    L.dgs_batch_plan_benefit.argtypes = [P, i32]
    L.dgs_batch_plan_benefit.restype = P
    L.dgs_batch_plan_assign.argtypes = [P, i32]
    L.dgs_batch_plan_assign.restype = P
    L.dgs_batch_plan_run.argtypes = [P, P, P, P]
    L.dgs_batch_plan_config.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.dgs_batch_plan_destroy.argtypes = [P]
    L.dgs_batch_plan_destroy.restype = None
    L.dgs_status_string.argtypes = [ctypes.c_int]
    L.dgs_status_string.restype = ctypes.c_char_p
    L.dgs_last_error.restype = ctypes.c_char_p
    L.dgs_version.restype = ctypes.c_char_p
    L.dgs_release_cached.restype = None
    for name in ("dgs_solve", "dgs_solve_ex", "dgs_solve_noalloc", "dgs_solve_batched", "dgs_diff_eval", "dgs_server_create",
                 "dgs_server_submit", "dgs_server_poll", "dgs_server_wait", "dgs_server_stats_get",
                 "dgs_batch_plan_create", "dgs_batch_plan_run", "dgs_batch_plan_config"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st: int, what: str):
    if st != DGS_OK:
        L = lib()
        msg = L.dgs_last_error().decode() or L.dgs_status_string(st).decode()
        raise DGSError(st, f"{what}: {msg}")


def _is_device_tensor(x) -> bool:
    return hasattr(x, "is_cuda") and bool(x.is_cuda)


def _host_i32(a, shape=None) -> np.ndarray:
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    a = np.ascontiguousarray(a, dtype=np.int32)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _square_n(A) -> int:
    shape = tuple(A.shape)
    if len(shape) != 2 or shape[0] != shape[1]:
        raise ValueError("benefit matrix must be square n x n")
    return int(shape[0])


def _torch_stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def solve(A, init=None, max_switches: int = -1, profile: bool = False, parallel: bool = False,
          lazy: bool = False, global_greedy: bool = False):
    """Run DGS on one instance.

    A: n x n int32 benefit matrix (numpy / CPU tensor, or a ROCm tensor).
    init: optional start permutation (same kind of memory as A).
    Returns (tau, result) with tau[i] the job of agent i (numpy for host
    inputs, a device tensor for device inputs) and result a dict.
    profile: also time each phase with HIP events (result["phase_ms"]).
    parallel: Parallel DGS (Algorithm 3 with Check Conflicts, Algorithm 4):
    every round applies all non-conflicting improving exchanges at once;
    max_switches then bounds the rounds (result["rounds"]).
    lazy: Algorithm 1 with stale stored bests (stale agent and job bests, the paper's
    branch rule and improvement guard); result["rounds"] = passes,
    result["attempts"] = exchanges tried.
    global_greedy: start from the global greedy assignment (largest
    remaining entry first) instead of the agent-order greedy one.
    """
    L = lib()
    n = _square_n(A)
    extra = ((DGS_PROFILE if profile else 0) | (DGS_PARALLEL if parallel else 0) | (DGS_LAZY if lazy else 0)
             | (DGS_GLOBAL_GREEDY if global_greedy else 0))
    opt = Options(max_switches=int(max_switches), init_assign=None, flags=extra, stream=None)
    res = Result()
    if _is_device_tensor(A):
        import torch
        if A.dtype != torch.int32 or not A.is_contiguous():
            raise ValueError("device benefit matrix must be contiguous int32")
        out = torch.empty(n, dtype=torch.int32, device=A.device)
        keep = None
        if init is not None:
            keep = init.to(device=A.device, dtype=torch.int32).contiguous()
            opt.init_assign = keep.data_ptr()
        opt.flags = DGS_DEVICE_PTRS | extra
        opt.stream = _torch_stream_ptr()
        st = L.dgs_solve_ex(A.data_ptr(), n, out.data_ptr(), ctypes.byref(opt), ctypes.byref(res))
        _check(st, "dgs_solve_ex")
        return out, res.as_dict()
    Ah = _host_i32(A)
    out = np.empty(n, dtype=np.int32)
    keep = None
    if init is not None:
        keep = _host_i32(init, (n,))
        opt.init_assign = keep.ctypes.data
    st = L.dgs_solve_ex(Ah.ctypes.data, n, out.ctypes.data, ctypes.byref(opt), ctypes.byref(res))
    _check(st, "dgs_solve_ex")
    return out, res.as_dict()


def solve_noalloc(A, out, init=None, max_switches: int = -1, profile: bool = False):
    """Steepest-ascent DGS with no allocation in the library (dgs_solve_noalloc).

    A: n x n contiguous int32 ROCm tensor (n <= NOALLOC_MAX_N); out: a
    contiguous int32 ROCm tensor of n entries that receives tau; init:
    optional start permutation (device tensor).  Runs on torch's current
    stream.  Returns the result dict.
    """
    L = lib()
    n = _square_n(A)
    opt = Options(max_switches=int(max_switches), init_assign=init.data_ptr() if init is not None else None,
                  flags=DGS_DEVICE_PTRS | (DGS_PROFILE if profile else 0), stream=_torch_stream_ptr())
    res = Result()
    st = L.dgs_solve_noalloc(A.data_ptr(), n, out.data_ptr(), ctypes.byref(opt), ctypes.byref(res))
    _check(st, "dgs_solve_noalloc")
    return res.as_dict()


def solve_rect(A, init=None, max_switches: int = -1, profile: bool = False, global_greedy: bool = False):
    """Steepest-ascent DGS on an n x m benefit matrix (n agents, m >= n jobs):
    swaps between agents and moves to unassigned jobs (dgs_solve_rect).

    A: n x m int32 (numpy / CPU tensor, or a ROCm tensor); init: optional n
    distinct jobs; global_greedy: start from the global greedy assignment.
    Returns (tau, result) as solve() does.
    """
    L = lib()
    shape = tuple(A.shape)
    if len(shape) != 2 or shape[0] > shape[1]:
        raise ValueError("benefit matrix must be n x m with n <= m")
    n, m = int(shape[0]), int(shape[1])
    opt = Options(max_switches=int(max_switches), init_assign=None,
                  flags=(DGS_PROFILE if profile else 0) | (DGS_GLOBAL_GREEDY if global_greedy else 0), stream=None)
    res = Result()
    if _is_device_tensor(A):
        import torch
        if A.dtype != torch.int32 or not A.is_contiguous():
            raise ValueError("device benefit matrix must be contiguous int32")
        out = torch.empty(n, dtype=torch.int32, device=A.device)
        keep = None
        if init is not None:
            keep = init.to(device=A.device, dtype=torch.int32).contiguous()
            opt.init_assign = keep.data_ptr()
        opt.flags |= DGS_DEVICE_PTRS
        opt.stream = _torch_stream_ptr()
        st = L.dgs_solve_rect(A.data_ptr(), n, m, out.data_ptr(), ctypes.byref(opt), ctypes.byref(res))
        _check(st, "dgs_solve_rect")
        return out, res.as_dict()
    Ah = np.ascontiguousarray(np.asarray(A), dtype=np.int32)
    out = np.empty(n, dtype=np.int32)
    keep = None
    if init is not None:
        keep = np.ascontiguousarray(np.asarray(init), dtype=np.int32).reshape(n)
        opt.init_assign = keep.ctypes.data
    st = L.dgs_solve_rect(Ah.ctypes.data, n, m, out.ctypes.data, ctypes.byref(opt), ctypes.byref(res))
    _check(st, "dgs_solve_rect")
    return out, res.as_dict()


def diff_eval(A, tau):
    """Difference evaluation of every agent for assignment tau.

    Returns (gain int64[n], job int32[n]); for n == 1, (INT64_MIN, -1).
    """
    L = lib()
    n = _square_n(A)
    res = Result()
    if _is_device_tensor(A):
        import torch
        t = tau.to(device=A.device, dtype=torch.int32).contiguous()
        g = torch.empty(n, dtype=torch.int64, device=A.device)
        j = torch.empty(n, dtype=torch.int32, device=A.device)
        opt = Options(max_switches=0, init_assign=None, flags=DGS_DEVICE_PTRS, stream=_torch_stream_ptr())
        st = L.dgs_diff_eval(A.data_ptr(), n, t.data_ptr(), g.data_ptr(), j.data_ptr(), ctypes.byref(opt),
                             ctypes.byref(res))
        _check(st, "dgs_diff_eval")
        return g, j
    Ah = _host_i32(A)
    t = _host_i32(tau, (n,))
    g = np.empty(n, dtype=np.int64)
    j = np.empty(n, dtype=np.int32)
    st = L.dgs_diff_eval(Ah.ctypes.data, n, t.ctypes.data, g.ctypes.data, j.ctypes.data, None, ctypes.byref(res))
    _check(st, "dgs_diff_eval")
    return g, j


def solve_batched(As: Sequence, max_switches: int = -1):
    """Solve many independent instances in one call.  Returns (taus, results)."""
    L = lib()
    count = len(As)
    if count == 0:
        return [], []
    device = _is_device_tensor(As[0])
    ns = np.array([_square_n(A) for A in As], dtype=np.int32)
    opt = Options(max_switches=int(max_switches), init_assign=None, flags=0, stream=None)
    results = (Result * count)()
    if device:
        import torch
        outs = [torch.empty(int(n), dtype=torch.int32, device=As[0].device) for n in ns]
        bptr = (ctypes.c_void_p * count)(*[A.data_ptr() for A in As])
        optr = (ctypes.c_void_p * count)(*[o.data_ptr() for o in outs])
        opt.flags = DGS_DEVICE_PTRS
        opt.stream = _torch_stream_ptr()
    else:
        hs = [_host_i32(A) for A in As]
        outs = [np.empty(int(n), dtype=np.int32) for n in ns]
        bptr = (ctypes.c_void_p * count)(*[h.ctypes.data for h in hs])
        optr = (ctypes.c_void_p * count)(*[o.ctypes.data for o in outs])
    st = L.dgs_solve_batched(count, bptr, ns.ctypes.data, optr, results, ctypes.byref(opt))
    _check(st, "dgs_solve_batched")
    return outs, [r.as_dict() for r in results]


class BatchPlan:
    """A fixed batch shape (sizes ns, each <= 2048) solved again and again.

    The plan owns the device buffers; run() replays one captured graph.
    autotune=True times both workgroup sizes of the batched solver on the
    first run and keeps the faster one.
    """

    def __init__(self, ns, max_switches: int = -1, autotune: bool = False):
        L = lib()
        self.ns = [int(n) for n in ns]
        arr = np.array(self.ns, dtype=np.int32)
        opt = Options(max_switches=int(max_switches), init_assign=None,
                      flags=DGS_AUTOTUNE if autotune else 0, stream=None)
        h = ctypes.c_void_p()
        _check(L.dgs_batch_plan_create(len(self.ns), arr.ctypes.data, ctypes.byref(opt), ctypes.byref(h)),
               "dgs_batch_plan_create")
        self._h = h

    def run(self, As=None, outs: bool = True):
        """Solve; As (host matrices) are copied in first when given.

        Returns (taus or None, results).
        """
        L = lib()
        count = len(self.ns)
        bptr = None
        if As is not None:
            hs = [_host_i32(A, (n, n)) for A, n in zip(As, self.ns)]
            bptr = (ctypes.c_void_p * count)(*[h.ctypes.data for h in hs])
        taus = None
        optr = None
        if outs:
            taus = [np.empty(n, dtype=np.int32) for n in self.ns]
            optr = (ctypes.c_void_p * count)(*[t.ctypes.data for t in taus])
        results = (Result * count)()
        _check(L.dgs_batch_plan_run(self._h, bptr, optr, results), "dgs_batch_plan_run")
        return taus, [r.as_dict() for r in results]

    def config(self):
        b = ctypes.c_int32()
        g = ctypes.c_int32()
        _check(lib().dgs_batch_plan_config(self._h, ctypes.byref(b), ctypes.byref(g)), "dgs_batch_plan_config")
        return int(b.value), int(g.value)

    def close(self):
        if self._h:
            lib().dgs_batch_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def release_cached() -> None:
    """Free the device memory the library caches between calls."""
    lib().dgs_release_cached()


def server_footprint(n: int) -> int:
    return int(lib().dgs_server_footprint(int(n)))


@dataclass
class _Pending:
    ticket: int
    n: int
    benefit: np.ndarray  # kept alive until completion


class Server:
    """Request loop: submit host instances, poll or wait for assignments."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 0, max_n: int = 0):
        L = lib()
        cfg = ServerConfig(int(hbm_budget_bytes), int(max_slots), int(max_n))
        h = ctypes.c_void_p()
        _check(L.dgs_server_create(ctypes.byref(cfg), ctypes.byref(h)), "dgs_server_create")
        self._h = h
        self._pending = {}

    def submit(self, A) -> int:
        Ah = _host_i32(A)
        n = _square_n(Ah)
        t = ctypes.c_uint64()
        _check(lib().dgs_server_submit(self._h, Ah.ctypes.data, n, ctypes.byref(t)), "dgs_server_submit")
        self._pending[int(t.value)] = _Pending(int(t.value), n, Ah)
        return int(t.value)

    def _finish(self, st, ticket, out, res):
        if st == DGS_E_AGAIN:
            return None
        self._pending.pop(ticket, None)
        _check(st, "dgs_server")
        return out, res.as_dict()

    def poll(self, ticket: int):
        """(tau, result) if done, else None."""
        p = self._pending.get(ticket)
        out = np.empty(p.n if p else 0, dtype=np.int32)
        res = Result()
        st = lib().dgs_server_poll(self._h, ticket, out.ctypes.data if p else None, ctypes.byref(res))
        return self._finish(st, ticket, out, res)

    def wait(self, ticket: int, timeout_us: int = -1):
        p = self._pending.get(ticket)
        out = np.empty(p.n if p else 0, dtype=np.int32)
        res = Result()
        st = lib().dgs_server_wait(self._h, ticket, out.ctypes.data if p else None, ctypes.byref(res),
                                   int(timeout_us))
        return self._finish(st, ticket, out, res)

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().dgs_server_stats_get(self._h, ctypes.byref(s)), "dgs_server_stats_get")
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            lib().dgs_server_destroy(self._h)
            self._h = None
            self._pending.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
