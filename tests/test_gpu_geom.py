"""GPU parity on the paper's GEOM instance type (Section 4): rounded
Euclidean distances of random points in a 1000 x 1000 square.

All three switching modes through the C ABI against the oracle, bit-exact.
At n = 16384 the expected values come from tests/golden/geom16384.txt,
written by tests/golden/make_golden.py --geom (oracle only).
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


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dgs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1106_5694_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("n", [2, 65, 256, 1000, 2048, 3000])
def test_steepest(dgs, n):
    A = gen.geom_matrix(n, 10 + n)
    say(f"geom steepest n={n}")
    tau, res = dgs.solve(A)
    ref = oracle.dgs_incr(A)
    assert (tau == ref["tau"]).all() and res["total_benefit"] == ref["f"] and res["switches"] == ref["S"]


@pytest.mark.parametrize("n", [2, 65, 256, 1000, 2048, 3000])
def test_parallel(dgs, n):
    A = gen.geom_matrix(n, 20 + n)
    say(f"geom parallel n={n}")
    tau, res = dgs.solve(A, parallel=True)
    ref = oracle.parallel_dgs(A)
    assert (tau == ref["tau"]).all() and res["total_benefit"] == ref["f"]
    assert res["switches"] == ref["S"] and res["rounds"] == ref["rounds"]


@pytest.mark.parametrize("n", [2, 65, 256, 1000, 2048])
def test_lazy(dgs, n):
    A = gen.geom_matrix(n, 30 + n)
    say(f"geom lazy n={n}")
    tau, res = dgs.solve(A, lazy=True)
    ref = oracle.lazy_dgs(A)
    assert (tau == ref["tau"]).all() and res["total_benefit"] == ref["f"]
    assert (res["switches"], res["attempts"], res["rounds"]) == (ref["S"], ref["attempts"], ref["passes"])


def test_random_start_all_modes(dgs):
    A = gen.geom_matrix(700, 4)
    init = gen.permutation(700, 4)
    say("geom random start n=700")
    t1, r1 = dgs.solve(A, init=init)
    assert (t1 == oracle.dgs_incr(A, init=init)["tau"]).all()
    t2, r2 = dgs.solve(A, init=init, parallel=True)
    assert (t2 == oracle.parallel_dgs(A, init=init)["tau"]).all()
    t3, r3 = dgs.solve(A, init=init, lazy=True)
    assert (t3 == oracle.lazy_dgs(A, init=init)["tau"]).all()
    assert r1["initial_benefit"] == r2["initial_benefit"] == r3["initial_benefit"] == oracle.objective(A, init)


@pytest.fixture(scope="module")
def geom16384():
    import torch
    return torch.from_numpy(gen.single_instance("geom16384", 1)).cuda()


@pytest.mark.parametrize("mode", ["steepest", "parallel", "lazy"])
def test_geom16384_golden(dgs, geom16384, mode):
    gold = read_sections(os.path.join(HERE, "golden", "geom16384.txt"))[f"{mode}_seed1"]
    say(f"geom16384 {mode}")
    A = geom16384
    tau, res = dgs.solve(A, parallel=mode == "parallel", lazy=mode == "lazy")
    h = hashlib.sha256(np.ascontiguousarray(tau.cpu().numpy(), dtype="<i4").tobytes()).hexdigest()
    assert res["initial_benefit"] == int(gold["greedy_f"])
    assert res["total_benefit"] == int(gold["f"]) and res["switches"] == int(gold["S"])
    if mode == "parallel":
        assert res["rounds"] == int(gold["rounds"])
    if mode == "lazy":
        assert res["attempts"] == int(gold["attempts"]) and res["rounds"] == int(gold["passes"])
    assert h == gold["tau_sha256"]


def test_batched_and_plan_on_geom(dgs):
    # the one-workgroup-per-instance solver on the paper's instance type:
    # sizes across its whole range, the largest beyond it (solved alone)
    ns = [2, 63, 64, 500, 1024, 2048, 2049, 3000]
    As = [gen.geom_matrix(n, 80 + i) for i, n in enumerate(ns)]
    say(f"geom batched: {ns}")
    refs = [oracle.dgs_incr(A) for A in As]
    taus, results = dgs.solve_batched(As)
    for ref, tau, res in zip(refs, taus, results):
        assert (tau == ref["tau"]).all() and res["total_benefit"] == ref["f"] and res["switches"] == ref["S"]
    small = [(A, ref) for A, ref in zip(As, refs) if A.shape[0] <= 2048]
    plan = dgs.BatchPlan([A.shape[0] for A, _ in small])
    try:
        for rep in range(3):  # replays of the captured graph, eager checks between them
            taus, results = plan.run([A for A, _ in small])
            for (A, ref), tau, res in zip(small, taus, results):
                assert (tau == ref["tau"]).all() and res["total_benefit"] == ref["f"], rep
    finally:
        plan.close()
