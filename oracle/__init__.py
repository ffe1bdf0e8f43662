"""CPU oracle for Deep Greedy Switching -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never imports, links or calls
it, and it shares no code with the GPU library: both sides only take their
inputs from ``workloads.gen``.

Contents:
  * ``dgs_ref``  -- pure-Python DGS from the definitions (tiny n).
  * ``brute``    -- exhaustive optimum (n <= 8).
  * ``oracle.c`` -- plain C DGS: greedy start, difference evaluation of
    every agent, DGS with a fresh full re-evaluation after every switch,
    DGS with exact incremental re-evaluation, and an O(n^3) Hungarian
    optimum.  Built by ``oracle/build.py`` into ``liboracle.so`` and
    wrapped below with ctypes.
  * ``parallel_dgs`` (below) -- Algorithm 3 with Check Conflicts
    (Algorithm 4): rounds of the C agent and job scans and an index-order
    claim walk over agents, then jobs.
  * ``rect_dgs`` (below) -- steepest-ascent DGS for n agents and m >= n
    jobs: swaps with other agents and moves to unassigned jobs, numpy;
    ``rect_dgs_full`` the same in C (``orc_rect_dgs``) for larger sizes,
    and ``global_greedy`` (``orc_global_greedy``) the global greedy start
    (largest remaining entry first).
  * ``lazy_dgs`` (below) -- lazy DGS, Algorithm 1 (stale stored bests of
    agents and jobs, the selection rule, the improvement guard, repeated
    passes), with numpy row evaluations.

Every function computes in int64.  Parity unpinned: none -- each function
is pinned by the tests listed in the repository's design notes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        L.orc_objective.restype = ctypes.c_int64
        L.orc_objective.argtypes = [i32p, ctypes.c_int32, i32p]
        L.orc_is_permutation.restype = ctypes.c_int32
        L.orc_is_permutation.argtypes = [i32p, ctypes.c_int32]
        L.orc_greedy.restype = None
        L.orc_greedy.argtypes = [i32p, ctypes.c_int32, i32p]
        L.orc_scan.restype = None
        L.orc_scan.argtypes = [i32p, ctypes.c_int32, i32p, i64p, i32p]
        L.orc_scan_jobs.restype = None
        L.orc_scan_jobs.argtypes = [i32p, ctypes.c_int32, i32p, i64p, i32p]
        L.orc_dgs_full.restype = ctypes.c_int64
        L.orc_dgs_full.argtypes = [i32p, ctypes.c_int32, i32p, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int64), i32p, i32p, i64p,
                                   ctypes.c_int64]
        L.orc_dgs_incr.restype = ctypes.c_int64
        L.orc_dgs_incr.argtypes = [i32p, ctypes.c_int32, i32p, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int64), i32p, i32p, i64p,
                                   ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.orc_set_threads.restype = ctypes.c_int32
        L.orc_set_threads.argtypes = [ctypes.c_int32]
        L.orc_global_greedy.restype = None
        L.orc_global_greedy.argtypes = [i32p, ctypes.c_int32, ctypes.c_int32, i32p]
        L.orc_rect_dgs.restype = ctypes.c_int64
        L.orc_rect_dgs.argtypes = [i32p, ctypes.c_int32, ctypes.c_int32, i32p, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int64)]
        L.orc_hungarian.restype = ctypes.c_int64
        L.orc_hungarian.argtypes = [i32p, ctypes.c_int32, i32p]
        _lib = L
    return _lib


NEG_INF = np.iinfo(np.int64).min


def _mat(A):
    A = np.ascontiguousarray(A, dtype=np.int32)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("benefit matrix must be square")
    return A


def set_threads(k: int) -> int:
    """OpenMP threads of the C oracle (k > 0); returns the count in effect."""
    return int(lib().orc_set_threads(int(k)))


def objective(A, tau):
    A = _mat(A)
    return int(lib().orc_objective(A, A.shape[0], np.ascontiguousarray(tau, dtype=np.int32)))


def is_permutation(tau):
    tau = np.ascontiguousarray(tau, dtype=np.int32)
    return bool(lib().orc_is_permutation(tau, tau.shape[0]))


def greedy(A):
    A = _mat(A)
    tau = np.empty(A.shape[0], dtype=np.int32)
    lib().orc_greedy(A, A.shape[0], tau)
    return tau


def scan(A, tau):
    """Per-agent best exchange (gain int64, job int32); NEG_INF/-1 when n == 1."""
    A = _mat(A)
    n = A.shape[0]
    g = np.empty(n, dtype=np.int64)
    j = np.empty(n, dtype=np.int32)
    lib().orc_scan(A, n, np.ascontiguousarray(tau, dtype=np.int32), g, j)
    return g, j


def scan_jobs(A, tau):
    """Per-job best exchange (gain int64, agent int32): the agent that would
    gain most by taking the job, its owner taking the agent's job; lowest
    agent on ties; NEG_INF/-1 when n == 1."""
    A = _mat(A)
    n = A.shape[0]
    g = np.empty(n, dtype=np.int64)
    i = np.empty(n, dtype=np.int32)
    lib().orc_scan_jobs(A, n, np.ascontiguousarray(tau, dtype=np.int32), g, i)
    return g, i


def _run(fn, A, init, max_switches, trace_cap, incremental):
    A = _mat(A)
    n = A.shape[0]
    tau = greedy(A) if init is None else np.array(init, dtype=np.int32, copy=True)
    f = ctypes.c_int64(0)
    cap = max(int(trace_cap), 0)
    ti = np.zeros(max(cap, 1), dtype=np.int32)
    tj = np.zeros(max(cap, 1), dtype=np.int32)
    tg = np.zeros(max(cap, 1), dtype=np.int64)
    if incremental:
        resc = ctypes.c_int64(0)
        S = fn(A, n, tau, int(max_switches), ctypes.byref(f), ti, tj, tg, cap, ctypes.byref(resc))
    else:
        resc = None
        S = fn(A, n, tau, int(max_switches), ctypes.byref(f), ti, tj, tg, cap)
    m = min(S, cap)
    out = dict(tau=tau, f=int(f.value), S=int(S),
               trace=(ti[:m].copy(), tj[:m].copy(), tg[:m].copy()))
    if resc is not None:
        out["rescans"] = int(resc.value)
    return out


def dgs_full(A, init=None, max_switches=-1, trace_cap=0):
    """DGS with a fresh re-evaluation of every agent after each switch."""
    return _run(lib().orc_dgs_full, A, init, max_switches, trace_cap, False)


def dgs_incr(A, init=None, max_switches=-1, trace_cap=0):
    """DGS with exact incremental re-evaluation (same result as dgs_full)."""
    return _run(lib().orc_dgs_incr, A, init, max_switches, trace_cap, True)


def _claim_in_order(pairs):
    """Walk candidate exchanges (pairs of agents) in the given order; keep a
    pair when neither agent is claimed by a pair kept before it, and claim
    both.  Returns the positions of the kept pairs."""
    claimed, kept = set(), []
    for pos, (x, y) in enumerate(pairs):
        if x not in claimed and y not in claimed:
            claimed.update((x, y))
            kept.append(pos)
    return kept


def check_conflicts(tau, ga, ja, gj, ij):
    """Check Conflicts (Algorithm 4) on one round's evaluations.  The
    positive agent exchanges (agent i to job ja[i], its owner to tau(i)) in
    agent order, then the positive job exchanges (agent ij[j] to job j, the
    owner of j to tau(ij[j])) in job order, each as its pair of agents, go
    through ``_claim_in_order``.  Returns (kept agent pairs [(i, partner)],
    kept job pairs [(new agent, owner)])."""
    n = len(tau)
    sigma = np.empty(n, dtype=np.int64)
    sigma[tau] = np.arange(n)
    agent_pairs = [(int(i), int(sigma[ja[i]])) for i in np.flatnonzero(ga > 0)]
    job_pairs = [(int(ij[j]), int(sigma[j])) for j in np.flatnonzero(gj > 0)]
    kept = _claim_in_order(agent_pairs + job_pairs)
    na = len(agent_pairs)
    return ([agent_pairs[p] for p in kept if p < na], [job_pairs[p - na] for p in kept if p >= na])


def parallel_dgs(A, init=None, max_rounds=-1):
    """Parallel DGS (Algorithm 3 with Check Conflicts, Algorithm 4): each
    round evaluates every agent (C scan) and every job (C job scan) afresh,
    keeps the exchanges ``check_conflicts`` lets through and applies them all
    (they share no agent, so each gain is exact and f grows by their sum).
    Stops when a round keeps nothing (no exchange improves f).
    Returns dict(tau, f, S = exchanges applied, rounds)."""
    A = _mat(A)
    tau = greedy(A) if init is None else np.array(init, dtype=np.int32, copy=True)
    S = rounds = 0
    while max_rounds < 0 or rounds < max_rounds:
        ga, ja = scan(A, tau)
        gj, ij = scan_jobs(A, tau)
        kept_a, kept_j = check_conflicts(tau, ga, ja, gj, ij)
        if not kept_a and not kept_j:
            break
        new = tau.copy()
        for x, y in kept_a + kept_j:
            new[x], new[y] = tau[y], tau[x]
        tau = new
        S += len(kept_a) + len(kept_j)
        rounds += 1
    return dict(tau=tau, f=objective(A, tau), S=S, rounds=rounds)


def _ade_row(A, tau, sigma, i):
    """Algorithm 2 for agent i: the best gain over jobs j != tau(i) of agent i
    taking j (its owner sigma(j) taking tau(i)), lowest job on ties; stored
    as (gain, job) when > 0, else (0, -1)."""
    n = A.shape[0]
    if n < 2:
        return 0, -1
    g = A[i, :] + A[sigma, tau[i]] - A[i, tau[i]] - A[sigma, np.arange(n)]
    g[tau[i]] = NEG_INF
    j = int(np.argmax(g))
    return (int(g[j]), j) if g[j] > 0 else (0, -1)


def _jde_row(A, tau, sigma, j):
    """The job side: the best gain over agents i != sigma(j) of agent i taking
    job j (sigma(j) taking tau(i)), lowest agent on ties; (gain, agent) when
    > 0, else (0, -1)."""
    n = A.shape[0]
    if n < 2:
        return 0, -1
    o = sigma[j]
    g = A[:, j] + A[o, tau] - A[np.arange(n), tau] - A[o, j]
    g[o] = NEG_INF
    i = int(np.argmax(g))
    return (int(g[i]), i) if g[i] > 0 else (0, -1)


class _StoredImprovements:
    """The stored improvements of lazy DGS (Section 3.3, Algorithm 1): for
    every agent its best exchange (ADE, Algorithm 2) and for every job its
    best exchange (the job side), kept only when the gain is positive, and
    left as they are until refreshed (so they may be stale)."""

    def __init__(self, A64, tau, sigma):
        n = A64.shape[0]
        self.A, self.n = A64, n
        self.agent = [_ade_row(A64, tau, sigma, i) for i in range(n)]   # (value, job)
        self.job = [_jde_row(A64, tau, sigma, j) for j in range(n)]     # (value, agent)
        self.va = np.array([v for v, _ in self.agent], dtype=np.int64)
        self.vj = np.array([v for v, _ in self.job], dtype=np.int64)

    def any_positive(self):
        return self.n > 1 and (self.va.max() > 0 or self.vj.max() > 0)

    def take(self):
        """The selection rule: the largest agent value and the largest job
        value (lowest index among equals on each side); the agent's exchange
        is followed only when its value is strictly larger.  The followed
        entry is cleared.  Returns the exchange as (agent, job)."""
        a, b = int(np.argmax(self.va)), int(np.argmax(self.vj))
        if self.va[a] > self.vj[b]:
            pair = (a, self.agent[a][1])
            self.va[a], self.agent[a] = 0, (0, -1)
        else:
            pair = (self.job[b][1], b)
            self.vj[b], self.job[b] = 0, (0, -1)
        return pair

    def refresh(self, tau, sigma, agents, jobs):
        for x in agents:
            self.agent[x] = _ade_row(self.A, tau, sigma, x)
            self.va[x] = self.agent[x][0]
        for y in jobs:
            self.job[y] = _jde_row(self.A, tau, sigma, y)
            self.vj[y] = self.job[y][0]


def lazy_dgs(A, init=None, max_switches=-1):
    """Lazy DGS (Section 3.3, Algorithm 1), numpy.  A pass stores the best
    positive improvement of every agent and every job
    (``_StoredImprovements``); exchanges are then taken in the selection
    order of ``_StoredImprovements.take`` until no stored value is positive.
    A taken exchange (agent i to job j, the current owner of j to i's job)
    is applied only if it raises f; after an applied one the two agents and
    the two jobs it moved are evaluated afresh, every other stored value
    stays as it was.  Passes repeat until one applies nothing; max_switches
    bounds the applied exchanges and is checked before every attempt.
    Returns dict(tau, f, S = switches applied, attempts, passes)."""
    A64 = _mat(A).astype(np.int64)
    n = A64.shape[0]
    tau = (greedy(A) if init is None else np.array(init, dtype=np.int32, copy=True)).astype(np.int64)
    sigma = np.empty(n, dtype=np.int64)
    S = attempts = passes = 0
    while max_switches < 0 or S < max_switches:
        passes += 1
        sigma[tau] = np.arange(n)
        stored = _StoredImprovements(A64, tau, sigma)
        applied = 0
        while stored.any_positive() and not (0 <= max_switches <= S):
            attempts += 1
            i, j = stored.take()
            k, t0 = int(sigma[j]), int(tau[i])
            if A64[i, j] + A64[k, t0] - A64[i, t0] - A64[k, j] <= 0:
                continue  # f would not rise: the exchange is dropped
            tau[i], tau[k] = j, t0
            sigma[j], sigma[t0] = i, k
            S += 1
            applied += 1
            stored.refresh(tau, sigma, (i, k), (j, t0))
        if applied == 0:
            break
    tau = tau.astype(np.int32)
    return dict(tau=tau, f=objective(A, tau), S=S, attempts=attempts, passes=passes)


def rect_greedy(A):
    """n x m (m >= n): agents in index order take their best free job, lowest
    job on ties."""
    A = np.asarray(A, dtype=np.int64)
    n, m = A.shape
    free = np.ones(m, dtype=bool)
    tau = np.empty(n, dtype=np.int64)
    for i in range(n):
        row = np.where(free, A[i], np.iinfo(np.int64).min)
        tau[i] = int(np.argmax(row))
        free[tau[i]] = False
    return tau


def rect_dgs(A, init=None, max_switches=-1):
    """Steepest-ascent DGS on an n x m benefit matrix (m >= n, the paper's n
    providers and m receivers): agent i may take any other job j; if j has an
    owner k, k takes tau(i) (a 2-exchange, gain a[i][j] + a[k][tau(i)] -
    a[i][tau(i)] - a[k][j]), else tau(i) becomes unassigned (gain a[i][j] -
    a[i][tau(i)]).  Each agent's best is the lowest job among its largest
    gains; the best agent (lowest index on ties) is applied while its gain is
    > 0, then every agent is evaluated afresh.  Returns dict(tau, f, S)."""
    A = np.asarray(A, dtype=np.int64)
    n, m = A.shape
    tau = rect_greedy(A) if init is None else np.array(init, dtype=np.int64, copy=True)
    S = 0
    rows = np.arange(n)
    while max_switches < 0 or S < max_switches:
        owner = np.full(m, -1, dtype=np.int64)
        owner[tau] = rows
        d = A[rows, tau]
        k = owner[None, :].repeat(n, 0)                       # owner of job j
        has = k >= 0
        kk = np.where(has, k, 0)
        back = np.where(has, A[kk, tau[:, None]] - A[kk, np.arange(m)[None, :]], 0)
        G = A - d[:, None] + back
        G[rows, tau] = np.iinfo(np.int64).min
        j = np.argmax(G, axis=1)
        g = G[rows, j]
        i = int(np.argmax(g))
        if g[i] <= 0:
            break
        jj = int(j[i])
        if owner[jj] >= 0:
            tau[owner[jj]] = tau[i]
        tau[i] = jj
        S += 1
    return dict(tau=tau.astype(np.int32), f=int(A[rows, tau].sum()), S=S)


def global_greedy(A):
    """n x m (n <= m): while an agent is free, the largest entry whose agent
    and job are both free is taken (lowest agent, then lowest job, on ties).
    C (sorted walk over all entries)."""
    A = np.ascontiguousarray(A, dtype=np.int32)
    n, m = A.shape
    if n > m:
        raise ValueError("need n <= m")
    tau = np.empty(n, dtype=np.int32)
    lib().orc_global_greedy(A, n, m, tau)
    return tau


def rect_dgs_full(A, init=None, max_switches=-1):
    """rect_dgs in C: every agent re-evaluated over all m jobs after every
    change (OpenMP over agents).  init: n distinct jobs (None: the greedy
    start of rect_greedy).  Returns dict(tau, f, S)."""
    A = np.ascontiguousarray(A, dtype=np.int32)
    n, m = A.shape
    tau = np.ascontiguousarray(rect_greedy(A) if init is None else init, dtype=np.int32).copy()
    f = ctypes.c_int64(0)
    S = lib().orc_rect_dgs(A, n, m, tau, int(max_switches), ctypes.byref(f))
    return dict(tau=tau, f=int(f.value), S=int(S))


def hungarian(A):
    """(optimal benefit, an optimal assignment)."""
    A = _mat(A)
    tau = np.empty(A.shape[0], dtype=np.int32)
    f = lib().orc_hungarian(A, A.shape[0], tau)
    return int(f), tau
