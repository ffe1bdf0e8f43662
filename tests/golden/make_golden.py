"""Write tests/golden/lowrank16384.txt from the CPU oracle alone.

For each seed of the n = 16384 low-rank-plus-noise workload this records
the oracle's greedy-start benefit, final benefit, switch count and the
SHA-256 of the final assignment (int32 little-endian).  The GPU tests
compare against these numbers because the oracle needs minutes at this
size.  Run from the repository root:

    python tests/golden/make_golden.py [seeds...]
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


if __name__ == "__main__":
    main([int(s) for s in sys.argv[1:]] or [1, 2, 3, 4, 5])
