"""Write tests/golden/lowrank16384.txt from the CPU oracle alone.

For each seed of the n = 16384 low-rank-plus-noise workload this records
the oracle's greedy-start benefit, final benefit, switch count and the
SHA-256 of the final assignment (int32 little-endian).  The GPU tests
compare against these numbers because the oracle needs minutes at this
size.  Run from the repository root:

    python tests/golden/make_golden.py [seeds...]

With ``--prefix`` it writes tests/golden/lowrank20480_prefix.txt instead:
the oracle's state after the first 1000 switches of the n = 20480 instance
(seed 1), a size whose switching launch gathers more than 8 exchange words
per thread.

With ``--parallel`` it writes tests/golden/lowrank16384_parallel.txt: the
oracle's Parallel DGS (Algorithm 3 with Check Conflicts) from the greedy
start of the n = 16384 workload, seeds 1 and 2.

With ``--geom`` it writes tests/golden/geom16384.txt: steepest-ascent DGS,
Parallel DGS and lazy DGS from the greedy start of the paper's GEOM instance
type at n = 16384 (workloads.gen.geom_matrix(16384, 1)).  ``--geom parallel``
(or any subset of steepest / parallel / lazy) rewrites only those sections.

With ``--full20480`` it writes tests/golden/lowrank20480.txt: the oracle's
complete runs (greedy start, to the end) of the n = 20480 instance (seed 1)
by steepest-ascent DGS -- the size whose switching launch gathers more than
8 exchange words per thread -- and by Parallel DGS, whose Check Conflicts
takes its walking variant above n = 16384.  ``--full20480 parallel`` (or
steepest) rewrites only that section.

With ``--rect`` it writes tests/golden/rect1000x16384.txt: rectangular
steepest-ascent DGS (the C oracle's rect_dgs_full) on the first 1000 rows of
the n = 16384 low-rank workload (1000 providers, 16384 receivers, seed 1),
from the agent-order greedy start and from the global greedy start.

With ``--lazy`` it writes tests/golden/lowrank16384_lazy.txt: the oracle's
lazy DGS (Algorithm 1 with stale stored bests) from the greedy start of the n = 16384
workload, seed 1.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads import gen  # noqa: E402

OUT = os.path.join(HERE, "lowrank16384.txt")
OUT_PREFIX = os.path.join(HERE, "lowrank20480_prefix.txt")
PREFIX_N, PREFIX_K = 20480, 1000
OUT_PARALLEL = os.path.join(HERE, "lowrank16384_parallel.txt")
OUT_LAZY = os.path.join(HERE, "lowrank16384_lazy.txt")
OUT_GEOM = os.path.join(HERE, "geom16384.txt")
OUT_FULL20480 = os.path.join(HERE, "lowrank20480.txt")
OUT_RECT = os.path.join(HERE, "rect1000x16384.txt")
RECT_N, RECT_M = 1000, 16384


def replace_sections(path, header, sections):
    """Write `sections` ({name: [lines]}) into the golden file at `path`,
    keeping every other section as it is (and `header` if the file is new)."""
    old, order, cur = {}, [], None
    head = list(header)
    if os.path.exists(path):
        head = []
        for line in open(path).read().splitlines():
            if line.startswith("[") and line.endswith("]"):
                cur = line[1:-1]
                order.append(cur)
                old[cur] = []
            elif cur is None:
                head.append(line)
            elif line:
                old[cur].append(line)
    for name, body in sections.items():
        if name not in old:
            order.append(name)
        old[name] = body
    out = [h for h in head if h]
    for name in order:
        out += ["", f"[{name}]"] + old[name]
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")


def main(seeds):
    lines = ["# Oracle results for the n = 16384 low-rank-plus-noise workload",
             "# (workloads.gen.lowrank_matrix(16384, seed)), written by make_golden.py",
             "# with the C oracle's incremental DGS (greedy start, run to the end).",
             "# tau_sha256 = SHA-256 of the final assignment as int32 little-endian."]
    for seed in seeds:
        t0 = time.time()
        A = gen.lowrank_matrix(16384, seed)
        g = oracle.greedy(A)
        f0 = oracle.objective(A, g)
        r = oracle.dgs_incr(A, init=g)
        h = hashlib.sha256(np.ascontiguousarray(r["tau"], dtype="<i4").tobytes()).hexdigest()
        lines += ["", f"[seed{seed}]", f"greedy_f = {f0}", f"f = {r['f']}", f"S = {r['S']}",
                  f"tau_sha256 = {h}"]
        print(f"seed {seed}: S={r['S']} f={r['f']} ({time.time() - t0:.0f} s)", flush=True)
        del A
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


def prefix(seed=1):
    t0 = time.time()
    A = gen.lowrank_matrix(PREFIX_N, seed)
    g = oracle.greedy(A)
    r = oracle.dgs_incr(A, init=g, max_switches=PREFIX_K)
    h = hashlib.sha256(np.ascontiguousarray(r["tau"], dtype="<i4").tobytes()).hexdigest()
    lines = [f"# Oracle state after the first {PREFIX_K} switches (greedy start) of the",
             f"# n = {PREFIX_N} low-rank-plus-noise workload (workloads.gen.lowrank_matrix({PREFIX_N}, seed)),",
             "# written by make_golden.py --prefix with the C oracle's incremental DGS.",
             "", f"[seed{seed}]", f"n = {PREFIX_N}", f"k = {PREFIX_K}", f"greedy_f = {oracle.objective(A, g)}",
             f"f = {r['f']}", f"S = {r['S']}", f"tau_sha256 = {h}"]
    with open(OUT_PREFIX, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"prefix seed {seed}: S={r['S']} f={r['f']} ({time.time() - t0:.0f} s)", flush=True)


def parallel(seeds=(1, 2)):
    lines = ["# Oracle Parallel DGS (Algorithm 3 with Check Conflicts, Algorithm 4) on the",
             "# n = 16384 low-rank-plus-noise workload (workloads.gen.lowrank_matrix(16384, seed)),",
             "# greedy start, run until no agent has an improving exchange; written by",
             "# make_golden.py --parallel.  tau_sha256 as in lowrank16384.txt."]
    for seed in seeds:
        t0 = time.time()
        A = gen.lowrank_matrix(16384, seed)
        g = oracle.greedy(A)
        r = oracle.parallel_dgs(A, init=g)
        h = hashlib.sha256(np.ascontiguousarray(r["tau"], dtype="<i4").tobytes()).hexdigest()
        lines += ["", f"[seed{seed}]", f"greedy_f = {oracle.objective(A, g)}", f"f = {r['f']}",
                  f"S = {r['S']}", f"rounds = {r['rounds']}", f"tau_sha256 = {h}"]
        print(f"parallel seed {seed}: S={r['S']} rounds={r['rounds']} f={r['f']} ({time.time() - t0:.0f} s)",
              flush=True)
        del A
    with open(OUT_PARALLEL, "w") as f:
        f.write("\n".join(lines) + "\n")


def lazy(seeds=(1,)):
    lines = ["# Oracle lazy DGS (Algorithm 1 with stale stored bests: stale agent and job bests, strict",
             "# branch rule, improvement guard, passes until one applies nothing) on the",
             "# n = 16384 low-rank-plus-noise workload (workloads.gen.lowrank_matrix(16384, seed)),",
             "# greedy start; written by make_golden.py --lazy.  tau_sha256 as in lowrank16384.txt."]
    for seed in seeds:
        t0 = time.time()
        A = gen.lowrank_matrix(16384, seed)
        g = oracle.greedy(A)
        r = oracle.lazy_dgs(A, init=g)
        h = hashlib.sha256(np.ascontiguousarray(r["tau"], dtype="<i4").tobytes()).hexdigest()
        lines += ["", f"[seed{seed}]", f"greedy_f = {oracle.objective(A, g)}", f"f = {r['f']}",
                  f"S = {r['S']}", f"attempts = {r['attempts']}", f"passes = {r['passes']}", f"tau_sha256 = {h}"]
        print(f"lazy seed {seed}: S={r['S']} attempts={r['attempts']} passes={r['passes']} f={r['f']} "
              f"({time.time() - t0:.0f} s)", flush=True)
        del A
    with open(OUT_LAZY, "w") as f:
        f.write("\n".join(lines) + "\n")


def geom(seed=1, modes=("steepest", "parallel", "lazy")):
    header = ["# Oracle results on the paper's GEOM instance type (Section 4) at n = 16384:",
              "# workloads.gen.geom_matrix(16384, seed), greedy start, run to the end, by",
              "# steepest-ascent DGS (oracle dgs_incr), Parallel DGS and lazy DGS; written by",
              "# make_golden.py --geom.  tau_sha256 as in lowrank16384.txt."]
    t0 = time.time()
    A = gen.geom_matrix(16384, seed)
    g = oracle.greedy(A)
    f0 = oracle.objective(A, g)
    runs = {"steepest": lambda: oracle.dgs_incr(A, init=g),
            "parallel": lambda: oracle.parallel_dgs(A, init=g),
            "lazy": lambda: oracle.lazy_dgs(A, init=g)}
    sections = {}
    for name in modes:
        r = runs[name]()
        h = hashlib.sha256(np.ascontiguousarray(r["tau"], dtype="<i4").tobytes()).hexdigest()
        body = [f"greedy_f = {f0}", f"f = {r['f']}", f"S = {r['S']}"]
        if "rounds" in r:
            body.append(f"rounds = {r['rounds']}")
        if "attempts" in r:
            body += [f"attempts = {r['attempts']}", f"passes = {r['passes']}"]
        body.append(f"tau_sha256 = {h}")
        sections[f"{name}_seed{seed}"] = body
        print(f"geom {name}: S={r['S']} f={r['f']} ({time.time() - t0:.0f} s)", flush=True)
    replace_sections(OUT_GEOM, header, sections)


def full20480(seed=1, modes=("steepest", "parallel")):
    header = [f"# Oracle results of complete runs (greedy start, to the end) on the n = {PREFIX_N}",
              f"# low-rank-plus-noise workload (workloads.gen.lowrank_matrix({PREFIX_N}, seed)), written by",
              "# make_golden.py --full20480: steepest-ascent DGS (the C oracle's incremental DGS) and",
              "# Parallel DGS.  tau_sha256 as in lowrank16384.txt."]
    t0 = time.time()
    A = gen.lowrank_matrix(PREFIX_N, seed)
    g = oracle.greedy(A)
    runs = {"steepest": lambda: oracle.dgs_incr(A, init=g), "parallel": lambda: oracle.parallel_dgs(A, init=g)}
    sections = {}
    for name in modes:
        r = runs[name]()
        h = hashlib.sha256(np.ascontiguousarray(r["tau"], dtype="<i4").tobytes()).hexdigest()
        body = [f"n = {PREFIX_N}", f"greedy_f = {oracle.objective(A, g)}", f"f = {r['f']}", f"S = {r['S']}"]
        if "rounds" in r:
            body.append(f"rounds = {r['rounds']}")
        body.append(f"tau_sha256 = {h}")
        sections[f"{name}_seed{seed}"] = body
        print(f"n={PREFIX_N} {name} seed {seed}: S={r['S']} f={r['f']} ({time.time() - t0:.0f} s)", flush=True)
    replace_sections(OUT_FULL20480, header, sections)


def rect(seed=1):
    header = [f"# Oracle results of rectangular steepest-ascent DGS (swaps and moves to unassigned jobs)",
              f"# on the first {RECT_N} rows of the n = {RECT_M} low-rank-plus-noise workload",
              f"# (workloads.gen.lowrank_matrix({RECT_M}, seed, rows={RECT_N})): {RECT_N} agents, {RECT_M} jobs,",
              "# run to the end from the agent-order greedy start (oracle.rect_dgs_full) and from",
              "# the global greedy start (oracle.global_greedy); written by make_golden.py --rect.",
              "# tau_sha256 as in lowrank16384.txt (the n agents' jobs)."]
    t0 = time.time()
    A = gen.lowrank_matrix(RECT_M, seed, rows=RECT_N)

    def sha(t):
        return hashlib.sha256(np.ascontiguousarray(t, dtype="<i4").tobytes()).hexdigest()

    sections = {}
    g = oracle.rect_greedy(A)
    r = oracle.rect_dgs_full(A, init=g)
    sections[f"greedy_seed{seed}"] = [f"start_f = {int(A[np.arange(RECT_N), g].sum())}", f"f = {r['f']}",
                                      f"S = {r['S']}", f"tau_sha256 = {sha(r['tau'])}"]
    print(f"rect greedy: S={r['S']} f={r['f']} ({time.time() - t0:.0f} s)", flush=True)
    gg = oracle.global_greedy(A)
    r = oracle.rect_dgs_full(A, init=gg)
    sections[f"global_seed{seed}"] = [f"start_f = {int(A[np.arange(RECT_N), gg].sum())}",
                                      f"start_sha256 = {sha(gg)}", f"f = {r['f']}", f"S = {r['S']}",
                                      f"tau_sha256 = {sha(r['tau'])}"]
    print(f"rect global greedy: S={r['S']} f={r['f']} ({time.time() - t0:.0f} s)", flush=True)
    replace_sections(OUT_RECT, header, sections)


if __name__ == "__main__":
    if sys.argv[1:2] == ["--prefix"]:
        prefix()
    elif sys.argv[1:2] == ["--parallel"]:
        parallel()
    elif sys.argv[1:2] == ["--lazy"]:
        lazy()
    elif sys.argv[1:2] == ["--geom"]:
        geom(modes=tuple(sys.argv[2:]) or ("steepest", "parallel", "lazy"))
    elif sys.argv[1:2] == ["--rect"]:
        rect()
    elif sys.argv[1:2] == ["--full20480"]:
        full20480(modes=tuple(sys.argv[2:]) or ("steepest", "parallel"))
    else:
        main([int(s) for s in sys.argv[1:]] or [1, 2, 3, 4, 5])
