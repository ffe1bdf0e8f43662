"""Exhaustive LSAP optimum for tiny instances (n <= 8).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Enumerates all n!
permutations (Section 3's problem statement taken literally) and returns
the maximum total benefit and the set of permutations reaching it.
"""
from __future__ import annotations

import itertools


def optimum(A):
    n = len(A)
    if n > 8:
        raise ValueError("brute force is for n <= 8")
    best, arg = None, []
    for perm in itertools.permutations(range(n)):
        f = sum(A[i][perm[i]] for i in range(n))
        if best is None or f > best:
            best, arg = f, [list(perm)]
        elif f == best:
            arg.append(list(perm))
    return best, arg
