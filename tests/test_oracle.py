"""Pins of the CPU oracle against facts that do not come from the oracle.

Each check names what fixes the expected value: a hand-worked example of
the paper's definitions (tests/golden/worked_examples.txt), a closed form,
brute-force enumeration, an independent library routine, or an
implementation written from a different statement of the same definition
(the pure-Python oracle evaluates every exchange by rebuilding the
assignment and re-summing the objective, with no gain algebra).
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest
import scipy.optimize

import oracle
from oracle import brute, dgs_ref
from tests.golden_io import ints, matrix, worked_examples
from workloads import gen

EX = worked_examples()


def _f(A, tau):
    return int(sum(int(A[i, tau[i]]) for i in range(len(tau))))


def _swap_gains_by_resumming(A, tau):
    """All 2-exchange gains, each by building the exchanged assignment."""
    n = len(tau)
    f0 = _f(A, tau)
    out = {}
    for i, k in itertools.combinations(range(n), 2):
        t = list(tau)
        t[i], t[k] = t[k], t[i]
        out[(i, k)] = _f(A, t) - f0
    return out


# ---- worked examples ----------------------------------------------------------------


@pytest.mark.parametrize("name", sorted(EX))
def test_worked_example_c_oracle(name):
    ex = EX[name]
    A = matrix(ex["A"])
    assert list(oracle.greedy(A)) == ints(ex["greedy"])
    assert oracle.objective(A, oracle.greedy(A)) == int(ex["greedy_f"])
    if "scan0_gain" in ex:
        g, j = oracle.scan(A, oracle.greedy(A))
        assert list(g) == ints(ex["scan0_gain"])
        assert list(j) == ints(ex["scan0_job"])
    for run in (oracle.dgs_full, oracle.dgs_incr):
        r = run(A)
        assert list(r["tau"]) == ints(ex["tau"]), name
        assert r["f"] == int(ex["f"])
        assert r["S"] == int(ex["S"])
    if "final_gain" in ex:
        g, j = oracle.scan(A, np.array(ints(ex["tau"]), dtype=np.int32))
        assert list(g) == ints(ex["final_gain"])
        assert list(j) == ints(ex["final_job"])
    assert oracle.hungarian(A)[0] == int(ex["opt"])
    assert brute.optimum(A.tolist())[0] == int(ex["opt"])


@pytest.mark.parametrize("name", sorted(EX))
def test_worked_example_python_oracle(name):
    ex = EX[name]
    A = matrix(ex["A"]).tolist()
    assert dgs_ref.greedy(A) == ints(ex["greedy"])
    if "scan0_gain" in ex:
        rb = dgs_ref.scan(A, dgs_ref.greedy(A))
        assert [g for g, _ in rb] == ints(ex["scan0_gain"])
        assert [j for _, j in rb] == ints(ex["scan0_job"])
    tau, f, S, _ = dgs_ref.dgs(A)
    assert tau == ints(ex["tau"]) and f == int(ex["f"]) and S == int(ex["S"])


def test_single_agent_scan_sentinel():
    g, j = oracle.scan(np.array([[3]], dtype=np.int32), np.array([0], dtype=np.int32))
    assert g[0] == oracle.NEG_INF and j[0] == -1


# ---- closed forms ------------------------------------------------------------------------


@pytest.mark.parametrize("n", [1, 2, 5, 64, 300])
def test_constant_matrix(n):
    # every permutation has the same benefit: identity by the tie rule, no switch
    A = np.full((n, n), 17, dtype=np.int32)
    r = oracle.dgs_full(A)
    assert list(r["tau"]) == list(range(n)) and r["S"] == 0 and r["f"] == 17 * n


@pytest.mark.parametrize("n,seed", [(3, 1), (50, 2), (257, 3)])
def test_separable_matrix(n, seed):
    # a_ij = r_i + c_j: all permutations tie, so every gain is 0 and no switch
    # happens; greedy takes columns in order of (c desc, j asc).
    r = gen.uniform_matrix(n, 0, 1000, seed)[:, 0]
    c = gen.uniform_matrix(n, 0, 50, seed + 100)[0]  # many equal c_j
    A = (r[:, None] + c[None, :]).astype(np.int32)
    expect = sorted(range(n), key=lambda j: (-int(c[j]), j))
    out = oracle.dgs_incr(A)
    assert list(out["tau"]) == expect and out["S"] == 0
    g, _ = oracle.scan(A, out["tau"])
    if n > 1:
        assert (g == 0).all()


@pytest.mark.parametrize("n,seed", [(2, 1), (7, 2), (100, 3), (1000, 4)])
def test_rank_one_matrix_reaches_rank_matching(n, seed):
    # a_ij = u_i * c_j, distinct positive u, c: exchange (i, k) gains
    # (u_i - u_k)(c_tau(k) - c_tau(i)), so the only 2-swap local optimum is the
    # matching of u and c by rank, which is also the optimum (rearrangement).
    rng_u = gen.permutation(4 * n, seed)[:n].astype(np.int64) + 1
    rng_c = gen.permutation(4 * n, seed + 7)[:n].astype(np.int64) + 1
    A = (rng_u[:, None] * rng_c[None, :]).astype(np.int32)
    out = oracle.dgs_incr(A)
    order_u = np.argsort(rng_u)
    order_c = np.argsort(rng_c)
    expect = np.empty(n, dtype=np.int64)
    expect[order_u] = order_c
    assert list(out["tau"]) == list(expect)
    assert out["f"] == int(np.sum(np.sort(rng_u) * np.sort(rng_c)))
    if n <= 100:
        assert oracle.dgs_full(A)["f"] == out["f"]


@pytest.mark.parametrize("n,seed", [(1, 1), (9, 2), (500, 3)])
def test_scaled_permutation_matrix(n, seed):
    pi = gen.permutation(n, seed)
    A = np.zeros((n, n), dtype=np.int32)
    A[np.arange(n), pi] = 1000
    out = oracle.dgs_full(A) if n < 100 else oracle.dgs_incr(A)
    assert list(out["tau"]) == list(pi) and out["S"] == 0 and out["f"] == 1000 * n


# ---- brute force and exact optimum -----------------------------------------------------


@pytest.mark.parametrize("seed", range(40))
def test_small_instances_against_brute_force(seed):
    n = 1 + seed % 8
    vmax = 3 if seed % 3 == 0 else 50  # heavy ties for every third seed
    A = gen.uniform_matrix(n, -vmax if seed % 5 == 0 else 0, vmax, 1000 + seed)
    opt, _ = brute.optimum(A.tolist())
    r = oracle.dgs_full(A, trace_cap=64)
    assert oracle.is_permutation(r["tau"])
    assert r["f"] == _f(A, r["tau"]) <= opt
    if n <= 2:
        assert r["f"] == opt
    # 2-swap local optimality at exit, every gain by re-summing
    assert max(_swap_gains_by_resumming(A, r["tau"]).values(), default=0) <= 0
    # every applied switch has gain > 0 and the recorded gain is the true
    # change of the objective
    tau = list(oracle.greedy(A))
    f = _f(A, tau)
    for i, j, g in zip(*r["trace"]):
        assert g > 0
        t2 = dgs_ref.switch(int(i), int(j), tau)
        assert _f(A, t2) - f == g
        tau, f = t2, _f(A, t2)
    assert tau == list(r["tau"])
    assert oracle.hungarian(A)[0] == opt


@pytest.mark.parametrize("n,seed", [(16, 1), (64, 2), (200, 3), (513, 4)])
def test_hungarian_matches_scipy(n, seed):
    A = gen.uniform_matrix(n, -500, 1000, seed)
    f, tau = oracle.hungarian(A)
    rows, cols = scipy.optimize.linear_sum_assignment(A.astype(np.int64), maximize=True)
    assert f == int(A[rows, cols].astype(np.int64).sum())
    assert oracle.is_permutation(tau) and _f(A, tau) == f


# ---- two statements of the same definition agree ----------------------------------------


@pytest.mark.parametrize("seed", range(60))
def test_python_and_c_oracles_agree(seed):
    n = [3, 4, 5, 6, 8, 11, 13, 16][seed % 8]
    lo, hi = [(0, 3), (0, 10), (-5, 5), (0, 1000)][seed % 4]
    A = gen.uniform_matrix(n, lo, hi, 5000 + seed)
    tau_p, f_p, S_p, tr_p = dgs_ref.dgs(A.tolist())
    for run in (oracle.dgs_full, oracle.dgs_incr):
        r = run(A, trace_cap=10_000)
        assert list(r["tau"]) == tau_p and r["f"] == f_p and r["S"] == S_p
        assert [tuple(int(x) for x in t) for t in zip(*r["trace"])] == tr_p
    g, j = oracle.scan(A, oracle.greedy(A))
    rb = dgs_ref.scan(A.tolist(), dgs_ref.greedy(A.tolist()))
    assert list(g) == [x for x, _ in rb] and list(j) == [y for _, y in rb]


@pytest.mark.parametrize("seed", range(12))
def test_full_and_incremental_agree(seed):
    n = [40, 97, 128, 255, 256, 300][seed % 6]
    if seed % 3 == 0:
        A = gen.uniform_matrix(n, 0, 4, 7000 + seed)  # many exact ties
    elif seed % 3 == 1:
        A = gen.lowrank_matrix(n, 7000 + seed)
    else:
        A = gen.uniform_matrix(n, -1000, 1000, 7000 + seed)
    a = oracle.dgs_full(A, trace_cap=100_000)
    b = oracle.dgs_incr(A, trace_cap=100_000)
    assert (a["tau"] == b["tau"]).all() and a["f"] == b["f"] and a["S"] == b["S"]
    for x, y in zip(a["trace"], b["trace"]):
        assert (x == y).all()


def test_random_start_and_resume():
    # the paper's random start (Section 3.1) and resuming from a prefix state:
    # steepest ascent depends only on the current assignment.
    A = gen.lowrank_matrix(300, 3)
    start = gen.permutation(300, 11)
    full = oracle.dgs_incr(A, init=start, trace_cap=100_000)
    assert full["S"] > 10
    for k in (0, 1, 5, full["S"] // 2, full["S"]):
        part = oracle.dgs_full(A, init=start, max_switches=k)
        assert part["S"] == k
        # the prefix state equals replaying the first k switches
        tau = list(start)
        for i, j in zip(full["trace"][0][:k], full["trace"][1][:k]):
            tau = dgs_ref.switch(int(i), int(j), tau)
        assert list(part["tau"]) == tau
        rest = oracle.dgs_incr(A, init=part["tau"])
        assert (rest["tau"] == full["tau"]).all() and rest["f"] == full["f"]
        assert rest["S"] == full["S"] - k


def test_objective_accounting():
    A = gen.uniform_matrix(256, 0, 1000, 1)
    r = oracle.dgs_full(A, trace_cap=10_000)
    f0 = oracle.objective(A, oracle.greedy(A))
    assert r["f"] == f0 + int(r["trace"][2].sum())
    assert (r["trace"][2] > 0).all()
    assert r["f"] <= oracle.hungarian(A)[0]


# ---- Parallel DGS (Algorithm 3 with Check Conflicts, Algorithm 4) ----------------------
# Worked by hand (identity start, every diagonal entry 10): agent 0's best exchange is
# with agent 1 (gain 1), agents 1 and 2 are each other's best (gain 10), agent 3 has no
# positive exchange.  Index order accepts agent 0 first (claiming 0 and 1); agents 1 and
# 2 conflict.  After (0, 1) the round-2 gains are all <= 0, so parallel DGS stops at
# tau = [1, 0, 2, 3], f = 41, one switch in one round; steepest ascent instead takes the
# gain-10 exchange (1, 2) and ends at f = 50.
PAR_A = [[10, 11, 5, 0],
         [10, 10, 15, 0],
         [5, 15, 10, 0],
         [0, 0, 0, 10]]


def test_parallel_worked_example():
    ident = [0, 1, 2, 3]
    r = oracle.parallel_dgs(np.array(PAR_A), init=ident)
    assert list(r["tau"]) == [1, 0, 2, 3] and r["f"] == 41 and r["S"] == 1 and r["rounds"] == 1
    assert dgs_ref.parallel_dgs(PAR_A, init=ident) == ([1, 0, 2, 3], 41, 1, 1)
    assert oracle.dgs_full(np.array(PAR_A), init=ident)["f"] == 50
    ka, kj, ca, cj = dgs_ref.check_conflicts(dgs_ref.scan(PAR_A, ident), dgs_ref.job_scan(PAR_A, ident), ident)
    assert ka == [(0, 1)] and kj == [] and ca == [1, 2] and cj == [0, 1, 2]


# Worked by hand: Check Conflicts' job half keeps an exchange that the agent half
# misses.  Start tau = [2, 3, 0, 1, 4], f = 1 + 7 + 18 + 4 + 20 = 50.
# Agent bests (gain, job), lowest job on ties: agent 0 (25, job 1; partner 3),
# agent 1 (11, job 2; partner 0), agent 2 (7, job 2; partner 0), agent 3 (25, job 2;
# partner 0), agent 4 (6, job 1; partner 3 -- job 3 with partner 1 also gains 6).
# Job bests (gain, agent), lowest agent on ties: job 0 (7, agent 0), job 1 (25, 0),
# job 2 (25, 3), job 3 (11, 0), job 4 (6, agent 1 -- agent 3 also gains 6; owner 4).
# Agent half: agent 0 is kept and claims {0, 3}; agents 1-4 each touch 0 or 3.
# Job half: jobs 0-3 touch 0 or 3; job 4 (agent 1 takes it, owner 4 takes job 3:
# 16 + 17 - 7 - 20 = 6) touches {1, 4}, unclaimed: kept.  Round 1 applies both,
# f = 50 + 25 + 6 = 81 at tau = [1, 4, 0, 2, 3]; round 2 finds no improving exchange.
CC5_A = [[8, 15, 1, 12, 3],
         [9, 13, 7, 7, 16],
         [18, 13, 18, 8, 0],
         [0, 4, 15, 4, 11],
         [2, 19, 7, 17, 20]]
CC5_TAU = [2, 3, 0, 1, 4]


def test_parallel_job_half_worked_example():
    rb, jb = dgs_ref.scan(CC5_A, CC5_TAU), dgs_ref.job_scan(CC5_A, CC5_TAU)
    assert rb == [(25, 1), (11, 2), (7, 2), (25, 2), (6, 1)]
    assert jb == [(7, 0), (25, 0), (25, 3), (11, 0), (6, 1)]
    ka, kj, ca, cj = dgs_ref.check_conflicts(rb, jb, CC5_TAU)
    assert ka == [(0, 3)] and kj == [(4, 1, 4)] and ca == [1, 2, 3, 4] and cj == [0, 1, 2, 3]
    assert dgs_ref.parallel_dgs(CC5_A, init=CC5_TAU) == ([1, 4, 0, 2, 3], 81, 2, 1)
    r = oracle.parallel_dgs(np.array(CC5_A), init=CC5_TAU)
    assert list(r["tau"]) == [1, 4, 0, 2, 3] and r["f"] == 81 and r["S"] == 2 and r["rounds"] == 1
    g, i = oracle.scan_jobs(np.array(CC5_A), CC5_TAU)
    assert list(g) == [7, 25, 25, 11, 6] and list(i) == [0, 0, 3, 0, 1]
    # the end is a 2-swap local optimum
    assert oracle.dgs_full(np.array(CC5_A), init=[1, 4, 0, 2, 3])["S"] == 0


@pytest.mark.parametrize("seed", range(12))
def test_job_scan_against_definition(seed):
    """The C job scan equals JDE by re-summing f (every agent taking the job)."""
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(1, 9))
    A = rng.integers(-6, 6 if seed % 2 else 3, (n, n))
    tau = [int(x) for x in rng.permutation(n)]
    g, i = oracle.scan_jobs(A, tau)
    for j in range(n):
        if n == 1:
            assert g[0] == oracle.NEG_INF and i[0] == -1
            continue
        ref = dgs_ref.jde(A.tolist(), tau, j)
        assert (int(g[j]), int(i[j])) == ref
        # brute force over agents, lowest agent among the largest gains
        gains = [(dgs_ref.objective(A.tolist(), dgs_ref.switch(a, j, tau)) - dgs_ref.objective(A.tolist(), tau), -a)
                 for a in range(n) if tau[a] != j]
        best = max(gains)
        assert (int(g[j]), int(i[j])) == (best[0], -best[1])


@pytest.mark.parametrize("name", ["2x2", "3x3 tie-break"])
def test_parallel_on_single_switch_examples(name):
    # one positive exchange per round: parallel DGS takes the same switches as DGS
    A = np.array({"2x2": [[5, 4], [4, 1]], "3x3 tie-break": [[9, 8, 8], [8, 1, 0], [8, 0, 1]]}[name])
    r, d = oracle.parallel_dgs(A), oracle.dgs_full(A)
    assert list(r["tau"]) == list(d["tau"]) and r["f"] == d["f"] and r["S"] == d["S"] == r["rounds"]


@pytest.mark.parametrize("seed", range(40))
def test_parallel_properties_small(seed):
    """Against the definitions: every round's kept exchanges are disjoint and
    positive, f grows by exactly their sum, no positive agent or job exchange
    is left that touches no claimed agent (the claims are maximal over both
    halves), the end is a 2-swap local optimum, the C-scan version equals the
    definitional one, and f <= the brute-force optimum."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 8))
    A = rng.integers(-20, 20 if seed % 2 else 3, (n, n))
    tau = list(dgs_ref.greedy(A.tolist())) if seed % 3 else [int(x) for x in rng.permutation(n)]
    start = list(tau)
    f = dgs_ref.objective(A.tolist(), tau)
    rounds = S = 0
    while True:
        rb, jb = dgs_ref.scan(A.tolist(), tau), dgs_ref.job_scan(A.tolist(), tau)
        ka, kj, ca, cj = dgs_ref.check_conflicts(rb, jb, tau)
        if not ka and not kj:
            assert all(g is None or g <= 0 for g, _ in rb) and all(g is None or g <= 0 for g, _ in jb)
            break
        sigma = dgs_ref.inverse(tau)
        pairs = list(ka) + [(i, o) for _, i, o in kj]
        used = [x for p in pairs for x in p]
        assert len(used) == len(set(used))  # disjoint
        claimed = set(used)
        for i, (g, j) in enumerate(rb):
            if g is not None and g > 0:
                assert {i, sigma[j]} & claimed  # maximal over the agent exchanges
        for j, (g, i) in enumerate(jb):
            if g is not None and g > 0:
                assert {i, sigma[j]} & claimed  # and over the job exchanges
        gain = sum(rb[i][0] for i, _ in ka) + sum(jb[j][0] for j, _, _ in kj)
        assert gain > 0
        for i, _ in ka:
            tau = dgs_ref.switch(i, rb[i][1], tau)
        for j, i, _ in kj:
            tau = dgs_ref.switch(i, j, tau)
        assert dgs_ref.objective(A.tolist(), tau) == f + gain
        f += gain
        rounds += 1
        S += len(pairs)
    r = oracle.parallel_dgs(A, init=start)
    assert list(r["tau"]) == tau and r["f"] == f and r["S"] == S and r["rounds"] == rounds
    assert r["f"] <= brute.optimum(A)[0]


def test_parallel_job_half_is_exercised():
    """On small tie-heavy instances the job half keeps exchanges the agent half
    cannot: the maximality check above is not vacuous for it."""
    rng = np.random.default_rng(77)
    hits = 0
    for _ in range(400):
        n = int(rng.integers(3, 8))
        A = rng.integers(0, 4, (n, n)).tolist()
        tau = [int(x) for x in rng.permutation(n)]
        _, kj, _, _ = dgs_ref.check_conflicts(dgs_ref.scan(A, tau), dgs_ref.job_scan(A, tau), tau)
        hits += bool(kj)
    assert hits >= 5


def test_parallel_prefix_and_resume():
    A = gen.uniform_matrix(300, 0, 1000, 3)
    full = oracle.parallel_dgs(A)
    part = oracle.parallel_dgs(A, max_rounds=2)
    rest = oracle.parallel_dgs(A, init=part["tau"])
    assert part["rounds"] == 2 and rest["rounds"] == full["rounds"] - 2
    assert list(rest["tau"]) == list(full["tau"]) and rest["f"] == full["f"]
    g, _ = oracle.scan(A, full["tau"])
    assert g.max() <= 0


# Lazy DGS (Algorithm 1 with stale stored bests), worked by hand from the identity start
# (f = 13).  Pass 1: stored agent bests (6, job 2), (5, job 0), (6, job 0) and
# job bests (6, agent 2), (5, agent 0), (6, agent 0) (job 1: agents 0 and 2
# tie at 5, the lower agent is kept).  Attempt 1: the maxima tie at 6 and the
# strict comparison takes the job branch: agent 2 takes job 0 (+6, f = 19);
# agents 0, 2 and jobs 0, 2 are re-evaluated: (1, job 1), (3, job 1) and
# (3, agent 1), (1, agent 1).  Attempt 2: stale maxima 5 and 5, job branch:
# agent 0 takes job 1 (+1, f = 20); agents 0, 1 and jobs 1, 2 fall to 0.
# Attempt 3: job 0's stale (3, agent 1) is now worth -2: not applied.
# Attempt 4: agent 2's stale (3, job 1) is worth -2: not applied.  Pass 2
# finds no improving exchange.  Steepest ascent reaches f = 22 instead.
LAZY_A = [[5, 5, 9], [7, 2, 7], [8, 6, 6]]


def test_lazy_worked_example():
    ident = [0, 1, 2]
    r = oracle.lazy_dgs(np.array(LAZY_A), init=ident)
    assert list(r["tau"]) == [1, 2, 0] and r["f"] == 20
    assert (r["S"], r["attempts"], r["passes"]) == (2, 4, 2)
    assert dgs_ref.lazy_dgs(LAZY_A, init=ident) == ([1, 2, 0], 20, 2, 4, 2)
    assert oracle.dgs_full(np.array(LAZY_A), init=ident)["f"] == 22
    # the stored bests of the first pass, from the definitions
    assert [dgs_ref.best_positive(dgs_ref.ade(LAZY_A, ident, i)) for i in range(3)] == [(6, 2), (5, 0), (6, 0)]
    assert [dgs_ref.best_positive(dgs_ref.jde(LAZY_A, ident, j)) for j in range(3)] == [(6, 2), (5, 0), (6, 0)]


@pytest.mark.parametrize("seed", range(60))
def test_lazy_matches_definitions_small(seed):
    """The numpy oracle against the definitional statement (every gain by
    re-summing f), plus what any run must satisfy: a permutation, every
    switch an improvement (f >= start), a 2-swap local optimum at the end
    (the last pass found nothing), f <= the brute-force optimum."""
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(1, 8))
    A = rng.integers(-20, 20 if seed % 3 else 3, (n, n))
    init = None if seed % 2 else list(rng.permutation(n))
    r = oracle.lazy_dgs(A, init=init)
    d = dgs_ref.lazy_dgs(A.tolist(), init=init)
    assert (list(r["tau"]), r["f"], r["S"], r["attempts"], r["passes"]) == (list(d[0]), d[1], d[2], d[3], d[4])
    start = dgs_ref.greedy(A.tolist()) if init is None else init
    assert r["f"] >= dgs_ref.objective(A.tolist(), start)
    assert r["attempts"] >= r["S"] and (r["passes"] >= 1)
    assert all(g is None or g <= 0 for g, _ in dgs_ref.scan(A.tolist(), list(r["tau"])))
    assert r["f"] <= brute.optimum(A.tolist())[0]


def test_lazy_two_agents_is_optimal():
    for A in ([[1, 5], [5, 1]], [[5, 1], [1, 5]], [[3, 3], [3, 3]], [[0, 7], [2, 0]]):
        r = oracle.lazy_dgs(np.array(A), init=[0, 1])
        assert r["f"] == brute.optimum(A)[0]


def test_lazy_anytime_prefix():
    A = gen.lowrank_matrix(200, 4)
    full = oracle.lazy_dgs(A)
    fs = []
    for k in range(0, 6):
        p = oracle.lazy_dgs(A, max_switches=k)
        assert p["S"] == min(k, full["S"])
        fs.append(p["f"])
    assert all(b > a for a, b in zip(fs, fs[1:]))
    assert oracle.lazy_dgs(A, max_switches=full["S"])["f"] == full["f"]


# Rectangular DGS (n agents, m > n jobs), worked by hand: greedy gives
# tau = [0, 2] (f = 7, job 1 free).  Both agents' best is their swap (+2);
# agent 0 wins the tie: tau = [2, 0], f = 9.  Then agent 0's best is the move
# to the free job 1 (+1): tau = [1, 0], f = 10, the optimum; nothing improves.
RECT_A = [[3, 1, 0], [9, 0, 4]]


def _rect_optimum(A):
    n, m = len(A), len(A[0])
    return max(sum(A[i][p[i]] for i in range(n)) for p in itertools.permutations(range(m), n))


def test_rect_worked_example():
    assert dgs_ref.rect_greedy(RECT_A) == [0, 2]
    r = oracle.rect_dgs(np.array(RECT_A))
    assert list(r["tau"]) == [1, 0] and r["f"] == 10 and r["S"] == 2
    assert dgs_ref.rect_dgs(RECT_A) == ([1, 0], 10, 2)
    assert oracle.rect_dgs(np.array(RECT_A), max_switches=1)["f"] == 9
    assert _rect_optimum(RECT_A) == 10


@pytest.mark.parametrize("seed", range(60))
def test_rect_matches_definitions_small(seed):
    """numpy oracle == definitional statement; no improving swap or move at
    the end; f <= the brute-force optimum over injective assignments."""
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(1, 5))
    m = int(rng.integers(n, n + 3))
    A = rng.integers(-9, 10 if seed % 3 else 3, (n, m))
    init = None if seed % 2 else [int(x) for x in rng.permutation(m)[:n]]
    r = oracle.rect_dgs(A, init=init)
    d = dgs_ref.rect_dgs(A.tolist(), init=init)
    assert (list(r["tau"]), r["f"], r["S"]) == (list(d[0]), d[1], d[2])
    L = A.tolist()
    tau = list(r["tau"])
    f = dgs_ref.rect_objective(L, tau)
    assert all(dgs_ref.rect_objective(L, dgs_ref.rect_switch(i, j, tau)) <= f
               for i in range(n) for j in range(m) if j != tau[i])
    assert r["f"] <= _rect_optimum(L)


def test_rect_square_is_steepest_ascent():
    for seed in range(10):
        A = gen.uniform_matrix(40, 0, 50 if seed % 2 else 4, 900 + seed)
        r, s = oracle.rect_dgs(A), oracle.dgs_full(A)
        assert list(r["tau"]) == list(s["tau"]) and r["f"] == s["f"] and r["S"] == s["S"]


# Global greedy start (largest remaining entry first), worked by hand.
# [[5, 9, 1], [2, 10, 3]]: the largest entry is 10 (agent 1, job 1); agent 0
# then takes its best free job, 0 (5): tau = [0, 1], f = 15.  The
# agent-order greedy gives tau = [1, 2] (9 + 3 = 12) instead.
GG_A = [[5, 9, 1], [2, 10, 3]]
# Ties: [[7, 0], [7, 5]] -- 7 twice in job 0: the lower agent 0 takes it,
# then agent 1 takes job 1 (f = 12; agent 1 first would give f = 7).
# [[7, 7], [0, 5]] -- 7 twice in agent 0: the lower job 0, then agent 1 takes
# job 1 (f = 12; job 1 first would give f = 7).
GG_TIES = [([[7, 0], [7, 5]], [0, 1]), ([[7, 7], [0, 5]], [0, 1])]


def test_global_greedy_worked_examples():
    assert dgs_ref.global_greedy(GG_A) == [0, 1]
    assert list(oracle.global_greedy(np.array(GG_A))) == [0, 1]
    assert dgs_ref.rect_greedy(GG_A) == [1, 2]
    for A, tau in GG_TIES:
        assert dgs_ref.global_greedy(A) == tau
        assert list(oracle.global_greedy(np.array(A))) == tau


@pytest.mark.parametrize("seed", range(80))
def test_global_greedy_matches_definition(seed):
    """The sorted walk (C) equals the repeated largest-entry definition on
    small instances with many ties, negative values and n <= m."""
    rng = np.random.default_rng(8100 + seed)
    n = int(rng.integers(1, 7))
    m = int(rng.integers(n, n + 5))
    A = rng.integers(-5, 6 if seed % 3 else 2, (n, m)).astype(np.int32)
    assert list(oracle.global_greedy(A)) == dgs_ref.global_greedy(A.tolist())


@pytest.mark.parametrize("n,m,seed", [(50, 50, 1), (40, 300, 2), (200, 210, 3)])
def test_global_greedy_rank_one_sorted_matching(n, m, seed):
    """Closed form: a_ij = u_i * c_j with distinct positive u and c -- the
    largest remaining entry always pairs the largest free u with the largest
    free c, so agents in decreasing u get the jobs of the n largest c in
    decreasing order."""
    rng = np.random.default_rng(seed)
    u = rng.permutation(np.arange(1, 4 * n + 1))[:n]
    c = rng.permutation(np.arange(1, 4 * m + 1))[:m]
    A = (u[:, None] * c[None, :]).astype(np.int32)
    tau = oracle.global_greedy(A)
    expect = np.empty(n, dtype=np.int64)
    expect[np.argsort(-u)] = np.argsort(-c)[:n]
    assert np.array_equal(tau, expect)


def test_global_greedy_half_of_optimum():
    """For nonnegative benefits the greedy matching is within a factor 2 of
    the optimum (every optimal pair loses to a taken entry at least as
    large on one of its two ends)."""
    for seed in range(20):
        A = gen.uniform_matrix(30, 0, 100, 300 + seed)
        f = oracle.objective(A, oracle.global_greedy(A))
        opt, _ = oracle.hungarian(A)
        assert 2 * f >= opt


@pytest.mark.parametrize("seed", range(30))
def test_rect_dgs_c_matches_numpy(seed):
    """orc_rect_dgs (C, full re-evaluation) == the numpy rect_dgs on random
    instances (ties, negatives, given starts, the global greedy start,
    prefixes)."""
    rng = np.random.default_rng(9100 + seed)
    n = int(rng.integers(1, 40))
    m = int(rng.integers(n, n + 60))
    A = rng.integers(-20, 20 if seed % 3 else 3, (n, m)).astype(np.int32)
    init = None
    if seed % 3 == 1:
        init = [int(x) for x in rng.permutation(m)[:n]]
    elif seed % 3 == 2:
        init = [int(x) for x in oracle.global_greedy(A)]
    ms = -1 if seed % 4 else int(rng.integers(0, 5))
    a = oracle.rect_dgs_full(A, init=init, max_switches=ms)
    b = oracle.rect_dgs(A, init=init, max_switches=ms)
    assert np.array_equal(a["tau"], b["tau"]) and a["f"] == b["f"] and a["S"] == b["S"]


def test_rect_from_global_greedy_worked_example():
    """GG_A from the global greedy start (tau = [0, 1], f = 15): agent 0's
    changes gain 1 - 5 (move to job 2) and 9 + 2 - 5 - 10 (swap); agent 1's
    move to job 2 gains 3 - 10 and its swap is the same: nothing improves.  From
    the agent-order start (tau = [1, 2], f = 12): agent 0's move to job 0
    gains 5 - 9, the swap 1 + 10 - 9 - 3 = -1, agent 1's move to job 0
    2 - 3: a local optimum at 12, below the global greedy start."""
    r = oracle.rect_dgs_full(np.array(GG_A, dtype=np.int32), init=oracle.global_greedy(np.array(GG_A)))
    assert list(r["tau"]) == [0, 1] and r["f"] == 15 and r["S"] == 0
    s = oracle.rect_dgs_full(np.array(GG_A, dtype=np.int32))
    assert list(s["tau"]) == [1, 2] and s["f"] == 12 and s["S"] == 0


def test_is_permutation_definition():
    """orc_is_permutation against the definition (the values are exactly
    0..n-1, each once) on hand-picked non-permutations -- a repeated value, a
    value n, a negative value, all equal -- and on random arrays, half of them
    permutations."""
    assert oracle.is_permutation([0]) and oracle.is_permutation([2, 0, 1])
    for bad in ([1], [-1], [0, 0], [1, 1], [0, 2], [3, 0, 1], [0, 1, -1], [2, 2, 2], [1, 2, 3]):
        assert not oracle.is_permutation(bad), bad
    rng = np.random.default_rng(11)
    for trial in range(200):
        n = int(rng.integers(1, 40))
        t = rng.permutation(n) if trial % 2 else rng.integers(-2, n + 2, size=n)
        assert oracle.is_permutation(t) == (sorted(int(x) for x in t) == list(range(n)))
