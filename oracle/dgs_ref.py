"""Pure-Python Deep Greedy Switching, written straight from the definitions.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Loops over Python
ints, for tiny instances: it is the first, most literal statement of what
the method computes, and it pins the C oracle (which must agree with it
exactly) on many small random instances.

  * objective f(sigma) = sum_i a[i][tau(i)]                   (Section 3)
  * switch(i, j, sigma): agent i takes job j, the old owner sigma(j) takes
    tau(i)                                                    (Section 3.3)
  * the gain of a switch is computed here by building the switched
    assignment and re-evaluating f from scratch -- not by a gain formula --
    so this oracle does not depend on any algebra about which terms cancel
  * ADE (Algorithm 2): scan jobs j' != tau(i) in index order, keep the
    first strictly better one
  * switching (Section 3.3, Algorithm 1) under steepest ascent: take the
    best switch over all agents (lowest agent on ties), apply it if its
    gain is > 0, re-evaluate every agent, repeat
  * greedy start (Section 3.1): agents in index order take their best free
    job, lowest index on ties
  * JDE (Section 3.3, job side of Algorithm 2): scan agents i' != sigma(j)
    in index order, keep the first strictly better one
  * Parallel DGS (Algorithm 3 with Check Conflicts, Algorithm 4): fresh
    agent and job evaluations per round, index-order claims of the two
    agents of every exchange (agents first, then jobs), all kept exchanges
    applied at once
  * rectangular DGS (n agents, m >= n jobs): steepest ascent over swaps
    with other agents and moves to unassigned jobs
  * lazy DGS (Algorithm 1 with stale stored bests): stale per-agent and per-job bests,
    the paper's branch rule and improvement guard, re-evaluation of the two
    agents and two jobs of an applied switch only, full passes repeated
    until a pass applies nothing
"""
from __future__ import annotations

NEG_INF = None  # marks "no other job" (n = 1)


def objective(A, tau):
    return sum(A[i][tau[i]] for i in range(len(tau)))


def inverse(tau):
    sigma = [-1] * len(tau)
    for i, j in enumerate(tau):
        sigma[j] = i
    return sigma


def switch(i, j, tau):
    """Return the assignment (as tau) after agent i takes job j."""
    sigma = inverse(tau)
    new = list(tau)
    k = sigma[j]
    j0 = tau[i]
    new[i] = j
    if k >= 0:
        new[k] = j0
    return new


def greedy(A):
    n = len(A)
    taken = [False] * n
    tau = []
    for i in range(n):
        best, bj = None, -1
        for j in range(n):
            if taken[j]:
                continue
            if best is None or A[i][j] > best:
                best, bj = A[i][j], j
        tau.append(bj)
        taken[bj] = True
    return tau


def ade(A, tau, i):
    """(gain, job) of agent i's best 2-exchange; (None, -1) if n == 1."""
    f0 = objective(A, tau)
    best, bj = NEG_INF, -1
    for jp in range(len(tau)):
        if jp == tau[i]:
            continue
        g = objective(A, switch(i, jp, tau)) - f0
        if best is None or g > best:
            best, bj = g, jp
    return best, bj


def scan(A, tau):
    return [ade(A, tau, i) for i in range(len(tau))]


def dgs(A, init=None, max_switches=-1):
    """Returns (tau, f, S, trace) with trace = [(agent, job, gain), ...]."""
    tau = list(greedy(A) if init is None else init)
    S = 0
    trace = []
    while max_switches < 0 or S < max_switches:
        rb = scan(A, tau)
        bi, bg = -1, 0
        for i, (g, _) in enumerate(rb):
            if g is not None and g > bg:
                bi, bg = i, g
        if bi < 0:
            break
        trace.append((bi, rb[bi][1], bg))
        tau = switch(bi, rb[bi][1], tau)
        S += 1
    return tau, objective(A, tau), S, trace


def claim_in_order(pairs):
    """Keep each pair of agents, in the given order, unless one of its two
    agents was claimed by a pair kept before it; a kept pair claims both.
    Returns a list of booleans (kept or not) for the pairs."""
    claimed, out = set(), []
    for x, y in pairs:
        ok = x not in claimed and y not in claimed
        if ok:
            claimed.update((x, y))
        out.append(ok)
    return out


def check_conflicts(rb, jb, tau):
    """Check Conflicts (Algorithm 4) over one round's fresh evaluations.

    rb[i] = (gain, job) of agent i's best exchange (ADE), jb[j] = (gain,
    agent) of job j's best exchange (JDE).  A positive agent exchange moves
    agent i to job j_i and the current owner sigma(j_i) to tau(i); a positive
    job exchange gives job j to agent i_j and moves the current owner sigma(j)
    to tau(i_j).  Either one involves exactly two agents.  The agent
    exchanges in agent order, then the job exchanges in job order, go through
    ``claim_in_order``: a conflict drops only the exchange that has it.

    Returns (kept agent exchanges [(i, partner)], kept job exchanges
    [(j, new agent, owner)], conflicting agents, conflicting jobs)."""
    sigma = inverse(tau)
    agents = [i for i, (g, _) in enumerate(rb) if g is not None and g > 0]
    jobs = [j for j, (g, _) in enumerate(jb) if g is not None and g > 0]
    pairs = [(i, sigma[rb[i][1]]) for i in agents] + [(jb[j][1], sigma[j]) for j in jobs]
    keep = claim_in_order(pairs)
    na = len(agents)
    kept_a = [pairs[p] for p in range(na) if keep[p]]
    conf_a = [agents[p] for p in range(na) if not keep[p]]
    kept_j = [(jobs[p - na], pairs[p][0], pairs[p][1]) for p in range(na, len(pairs)) if keep[p]]
    conf_j = [jobs[p - na] for p in range(na, len(pairs)) if not keep[p]]
    return kept_a, kept_j, conf_a, conf_j


def job_scan(A, tau):
    return [jde(A, tau, j) for j in range(len(tau))]


def parallel_dgs(A, init=None, max_rounds=-1):
    """Parallel DGS (Algorithm 3): every round evaluates every agent and every
    job afresh, keeps the exchanges Check Conflicts lets through and applies
    them all at once (they share no agent, so each gain is exact and f grows
    by their sum).  Rounds repeat until none is kept, which happens exactly
    when no exchange improves f.  Returns (tau, f, switches, rounds)."""
    tau = list(greedy(A) if init is None else init)
    S = rounds = 0
    while max_rounds < 0 or rounds < max_rounds:
        rb, jb = scan(A, tau), job_scan(A, tau)
        kept_a, kept_j, _, _ = check_conflicts(rb, jb, tau)
        if not kept_a and not kept_j:
            break
        new = list(tau)
        for i, p in kept_a:
            new[i], new[p] = tau[p], tau[i]
        for _, i, o in kept_j:
            new[i], new[o] = tau[o], tau[i]
        tau = new
        S += len(kept_a) + len(kept_j)
        rounds += 1
    return tau, objective(A, tau), S, rounds


def best_positive(pair):
    """Algorithm 2 keeps the start assignment unless a strictly better one
    exists: the stored improvement is the best gain if > 0, else 0."""
    g, x = pair
    return (g, x) if g is not None and g > 0 else (0, -1)


def jde(A, tau, j):
    """(gain, agent) of job j's best 2-exchange: agent i' != sigma(j) takes j
    (its old owner takes tau(i')); first strictly better agent in index order."""
    f0 = objective(A, tau)
    owner = inverse(tau)[j]
    best, bi = NEG_INF, -1
    for ip in range(len(tau)):
        if ip == owner:
            continue
        g = objective(A, switch(ip, j, tau)) - f0
        if best is None or g > best:
            best, bi = g, ip
    return best, bi


def stored_improvements(A, tau):
    """Lazy DGS's stored values (Section 3.3, Algorithm 1): every agent's and
    every job's best exchange, positive improvements only."""
    n = len(A)
    return ([best_positive(ade(A, tau, i)) for i in range(n)],
            [best_positive(jde(A, tau, j)) for j in range(n)])


def take_stored(agent_vals, job_vals):
    """The selection rule: the largest agent value and the largest job value
    (lowest index on ties on each side); the agent's exchange only when its
    value is strictly larger.  Clears the entry taken and returns the exchange
    as (agent, job)."""
    n = len(agent_vals)
    a = max(range(n), key=lambda i: (agent_vals[i][0], -i))
    b = max(range(n), key=lambda j: (job_vals[j][0], -j))
    if agent_vals[a][0] > job_vals[b][0]:
        pair = (a, agent_vals[a][1])
        agent_vals[a] = (0, -1)
    else:
        pair = (job_vals[b][1], b)
        job_vals[b] = (0, -1)
    return pair


def lazy_dgs(A, init=None, max_switches=-1):
    """Lazy DGS (Section 3.3, Algorithm 1): passes of stored improvements
    taken in the selection order, each exchange applied only when it raises
    f, the two agents and two jobs of an applied exchange evaluated afresh.
    Returns (tau, f, S, attempts, passes)."""
    n = len(A)
    tau = list(greedy(A) if init is None else init)
    S = attempts = passes = 0
    while max_switches < 0 or S < max_switches:
        passes += 1
        agent_vals, job_vals = stored_improvements(A, tau)
        applied = 0
        while max(v for v, _ in agent_vals + job_vals) > 0 and not (0 <= max_switches <= S):
            attempts += 1
            i, j = take_stored(agent_vals, job_vals)
            k, t0 = inverse(tau)[j], tau[i]
            new = switch(i, j, tau)
            if objective(A, new) <= objective(A, tau):
                continue
            tau = new
            S += 1
            applied += 1
            for x in (i, k):
                agent_vals[x] = best_positive(ade(A, tau, x))
            for y in (j, t0):
                job_vals[y] = best_positive(jde(A, tau, y))
        if applied == 0:
            break
    return tau, objective(A, tau), S, attempts, passes


def rect_objective(A, tau):
    return sum(A[i][tau[i]] for i in range(len(tau)))


def rect_greedy(A):
    """Agents in index order take their best free job, lowest job on ties."""
    m = len(A[0])
    taken = [False] * m
    tau = []
    for row in A:
        best, bj = None, -1
        for j in range(m):
            if not taken[j] and (best is None or row[j] > best):
                best, bj = row[j], j
        tau.append(bj)
        taken[bj] = True
    return tau


def global_greedy(A):
    """While an agent is free: among all entries whose agent and job are both
    free, take a largest one (the lowest agent, then the lowest job, among
    equal entries)."""
    n, m = len(A), len(A[0])
    tau = [-1] * n
    job_free = [True] * m
    for _ in range(n):
        best = None
        for i in range(n):
            if tau[i] >= 0:
                continue
            for j in range(m):
                if job_free[j] and (best is None or A[i][j] > best[0]):
                    best = (A[i][j], i, j)
        _, i, j = best
        tau[i] = j
        job_free[j] = False
    return tau


def rect_switch(i, j, tau):
    """Agent i takes job j; its owner, if any, takes tau(i); else the old job of
    i becomes unassigned."""
    new = list(tau)
    if j in new:
        new[new.index(j)] = tau[i]
    new[i] = j
    return new


def rect_dgs(A, init=None, max_switches=-1):
    """Steepest ascent on the rectangular neighbourhood: every agent's best
    change (first strictly better job in index order, gains by re-summing f),
    the best agent (lowest index on ties) applied while its gain is > 0.
    Returns (tau, f, S)."""
    m = len(A[0])
    tau = list(rect_greedy(A) if init is None else init)
    S = 0
    while max_switches < 0 or S < max_switches:
        f0 = rect_objective(A, tau)
        bi, bj, bg = -1, -1, 0
        for i in range(len(tau)):
            best, jb = None, -1
            for j in range(m):
                if j == tau[i]:
                    continue
                g = rect_objective(A, rect_switch(i, j, tau)) - f0
                if best is None or g > best:
                    best, jb = g, j
            if best is not None and best > bg:
                bi, bj, bg = i, jb, best
        if bi < 0:
            break
        tau = rect_switch(bi, bj, tau)
        S += 1
    return tau, rect_objective(A, tau), S
