"""GPU parity of lazy DGS (Algorithm 1 with stale stored bests).

The HIP path (dgs_solve_ex with DGS_LAZY, through the C ABI) against
oracle.lazy_dgs, bit-exact: the same assignment, total benefit, switches,
attempts and passes.  At n = 16384 the expected values come from
tests/golden/lowrank16384_lazy.txt, written by tests/golden/make_golden.py
--lazy (oracle only).
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np
import pytest

import oracle
from tests.golden_io import read_sections
from workloads import gen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))

# Worked by hand in tests/test_oracle.py: two job-branch switches, two stale
# attempts that fail the guard, a second pass that finds nothing.
LAZY_A = np.array([[5, 5, 9], [7, 2, 7], [8, 6, 6]], dtype=np.int32)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dgs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1106_5694_amd as m
    m.lib()
    return m


def check(dgs, A, init=None, max_switches=-1, what=""):
    say(f"lazy case {what}: n={A.shape[0]} init={'yes' if init is not None else 'greedy'} k={max_switches}")
    tau, res = dgs.solve(A, init=init, max_switches=max_switches, lazy=True)
    ref = oracle.lazy_dgs(A, init=init, max_switches=max_switches)
    assert oracle.is_permutation(tau)
    assert (tau == ref["tau"]).all(), what
    assert res["total_benefit"] == ref["f"] == oracle.objective(A, tau), what
    assert res["switches"] == ref["S"], what
    assert res["attempts"] == ref["attempts"], what
    assert res["rounds"] == ref["passes"], what
    return tau, res


def test_worked_example(dgs):
    tau, res = dgs.solve(LAZY_A, init=np.arange(3, dtype=np.int32), lazy=True)
    assert list(tau) == [1, 2, 0]
    assert (res["total_benefit"], res["switches"], res["attempts"], res["rounds"]) == (20, 2, 4, 2)
    assert res["initial_benefit"] == 13


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_uniform256(dgs, seed):
    check(dgs, gen.single_instance("uniform256", seed), what=f"uniform256 seed {seed}")


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 127, 1023, 1025])
@pytest.mark.parametrize("kind", ["ties", "signed", "lowrank"])
def test_edge_sizes(dgs, n, kind):
    if kind == "ties":
        A = gen.uniform_matrix(n, 0, 3, 100 + n)
    elif kind == "signed":
        A = gen.uniform_matrix(n, -1000, 1000, 200 + n)
    else:
        A = gen.lowrank_matrix(n, 300 + n)
    check(dgs, A, what=f"{kind} n={n}")


def test_extreme_values(dgs):
    m = (1 << 29) - 1
    rng = np.random.default_rng(6)
    A = rng.choice(np.array([-m, m, 0, 1 - m, m - 1], dtype=np.int32), size=(300, 300)).astype(np.int32)
    check(dgs, A, what="extreme values n=300")


@pytest.mark.parametrize("n", [500, 2049])
def test_random_start(dgs, n):
    A = gen.lowrank_matrix(n, 50 + n)
    init = np.random.default_rng(n + 1).permutation(n).astype(np.int32)
    check(dgs, A, init=init, what=f"random start n={n}")


@pytest.mark.parametrize("k", [0, 1, 7, 100])
def test_anytime_prefix(dgs, k):
    check(dgs, gen.lowrank_matrix(700, 12), max_switches=k, what=f"prefix of {k} switches")


def test_lowrank4096(dgs):
    check(dgs, gen.lowrank_matrix(4096, 9), what="lowrank n=4096")


def test_limits(dgs):
    with pytest.raises(dgs.DGSError) as e:
        dgs.solve(np.zeros((16385, 16385), dtype=np.int32), lazy=True)
    assert e.value.status == dgs.DGS_E_INVAL
    with pytest.raises(dgs.DGSError) as e:
        dgs.solve(gen.uniform_matrix(64, 0, 10, 1), lazy=True, parallel=True)
    assert e.value.status == dgs.DGS_E_INVAL
    A = gen.uniform_matrix(100, 0, 1000, 1)
    A[3, 7] = -(1 << 29)
    with pytest.raises(dgs.DGSError) as e:
        dgs.solve(A, lazy=True)
    assert e.value.status == dgs.DGS_E_RANGE
    check(dgs, gen.uniform_matrix(100, 0, 1000, 2), what="after errors")


def test_lowrank16384_golden(dgs):
    gold = read_sections(os.path.join(HERE, "golden", "lowrank16384_lazy.txt"))["seed1"]
    say("lazy case lowrank16384 seed 1")
    A = gen.lowrank_matrix(16384, 1)
    tau, res = dgs.solve(A, lazy=True)
    h = hashlib.sha256(np.ascontiguousarray(tau, dtype="<i4").tobytes()).hexdigest()
    assert res["initial_benefit"] == int(gold["greedy_f"])
    assert res["total_benefit"] == int(gold["f"])
    assert res["switches"] == int(gold["S"]) and res["attempts"] == int(gold["attempts"])
    assert res["rounds"] == int(gold["passes"])
    assert h == gold["tau_sha256"]
