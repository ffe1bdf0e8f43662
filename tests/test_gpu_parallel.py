"""GPU parity of Parallel DGS (Algorithm 3 with Check Conflicts, Algorithm 4).

The HIP path (dgs_solve_ex with DGS_PARALLEL, through the C ABI) against
oracle.parallel_dgs, bit-exact: the same assignment, total benefit,
number of exchanges applied and number of rounds.  At n = 16384 the
expected values come from tests/golden/lowrank16384_parallel.txt, written
by tests/golden/make_golden.py --parallel (oracle only).
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

# Identity start: agent 0's best exchange (with agent 1) is accepted first
# and claims agents 0 and 1, so agent 1's and agent 2's better exchanges
# (both with a claimed agent) are conflicts; one round, one exchange.
PAR_A = np.array([[10, 11, 5, 0], [10, 10, 15, 0], [5, 15, 10, 0], [0, 0, 0, 10]], dtype=np.int32)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dgs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1106_5694_amd as m
    m.lib()
    return m


def check(dgs, A, init=None, max_rounds=-1, what=""):
    say(f"parallel case {what}: n={A.shape[0]} init={'yes' if init is not None else 'greedy'} rounds<={max_rounds}")
    tau, res = dgs.solve(A, init=init, max_switches=max_rounds, parallel=True)
    ref = oracle.parallel_dgs(A, init=init, max_rounds=max_rounds)
    assert oracle.is_permutation(tau)
    assert (tau == ref["tau"]).all(), what
    assert res["total_benefit"] == ref["f"] == oracle.objective(A, tau), what
    assert res["switches"] == ref["S"], what
    assert res["rounds"] == ref["rounds"], what
    return tau, res


# Check Conflicts' job half (worked by hand in tests/test_oracle.py): from
# tau = [2, 3, 0, 1, 4] (f = 50) round 1 keeps agent 0's exchange with agent 3
# (+25) and job 4's exchange (agent 1 takes it, owner 4 takes job 3; +6), which
# the agent half cannot keep (agent 4's best, tied with it, is towards agent 3).
CC5_A = np.array([[8, 15, 1, 12, 3], [9, 13, 7, 7, 16], [18, 13, 18, 8, 0], [0, 4, 15, 4, 11],
                  [2, 19, 7, 17, 20]], dtype=np.int32)


def test_job_half_worked_example(dgs):
    tau, res = dgs.solve(CC5_A, init=np.array([2, 3, 0, 1, 4], dtype=np.int32), parallel=True)
    assert list(tau) == [1, 4, 0, 2, 3]
    assert res["initial_benefit"] == 50 and res["total_benefit"] == 81
    assert res["switches"] == 2 and res["rounds"] == 1
    # one round bounded: the same state
    tau1, res1 = dgs.solve(CC5_A, init=np.array([2, 3, 0, 1, 4], dtype=np.int32), max_switches=1, parallel=True)
    assert list(tau1) == [1, 4, 0, 2, 3] and res1["switches"] == 2


def test_worked_example_conflicts(dgs):
    tau, res = dgs.solve(PAR_A, init=np.arange(4, dtype=np.int32), parallel=True)
    assert list(tau) == [1, 0, 2, 3]
    assert res["total_benefit"] == 41 and res["switches"] == 1 and res["rounds"] == 1
    assert res["initial_benefit"] == 40


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_uniform256(dgs, seed):
    check(dgs, gen.single_instance("uniform256", seed), what=f"uniform256 seed {seed}")


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 127, 129, 257, 1000])
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
    rng = np.random.default_rng(5)
    A = rng.choice(np.array([-m, m, 0, 1 - m, m - 1], dtype=np.int32), size=(300, 300)).astype(np.int32)
    check(dgs, A, what="extreme values n=300")


@pytest.mark.parametrize("n", [500, 2049])
def test_random_start(dgs, n):
    A = gen.lowrank_matrix(n, 40 + n)
    init = np.random.default_rng(n).permutation(n).astype(np.int32)
    check(dgs, A, init=init, what=f"random start n={n}")


def test_lowrank4096(dgs):
    check(dgs, gen.lowrank_matrix(4096, 9), what="lowrank n=4096")


@pytest.mark.parametrize("k", [0, 1, 2, 5])
def test_round_prefix_and_resume(dgs, k):
    A = gen.lowrank_matrix(1500, 77)
    tau_k, res_k = check(dgs, A, max_rounds=k, what=f"prefix of {k} rounds")
    assert res_k["rounds"] == min(k, oracle.parallel_dgs(A)["rounds"])
    # every round starts from a fresh evaluation, so resuming from the prefix
    # ends where the uninterrupted run ends
    tau_r, res_r = dgs.solve(A, init=tau_k, parallel=True)
    full = oracle.parallel_dgs(A)
    assert (tau_r == full["tau"]).all()
    assert res_r["rounds"] == full["rounds"] - res_k["rounds"]
    assert res_k["switches"] + res_r["switches"] == full["S"]


def test_ends_at_local_optimum(dgs):
    A = gen.lowrank_matrix(3000, 11)
    tau, res = dgs.solve(A, parallel=True)
    g, _ = oracle.scan(A, tau)
    assert (g <= 0).all()
    assert res["total_benefit"] >= res["initial_benefit"]


def test_device_pointers(dgs):
    import torch
    A = gen.lowrank_matrix(700, 3)
    ref = oracle.parallel_dgs(A)
    tau, res = dgs.solve(torch.from_numpy(A).cuda(), parallel=True)
    assert (tau.cpu().numpy() == ref["tau"]).all()
    assert res["total_benefit"] == ref["f"] and res["rounds"] == ref["rounds"]


def test_range_error(dgs):
    A = gen.uniform_matrix(100, 0, 1000, 1)
    A[7, 3] = 1 << 29
    with pytest.raises(dgs.DGSError) as e:
        dgs.solve(A, parallel=True)
    assert e.value.status == dgs.DGS_E_RANGE
    # the library stays usable
    check(dgs, gen.uniform_matrix(100, 0, 1000, 2), what="after range error")


def test_sequential_mode_reports_no_rounds(dgs):
    _, res = dgs.solve(gen.single_instance("uniform256", 1))
    assert res["rounds"] == 0


@pytest.mark.parametrize("seed", [1, 2])
def test_lowrank16384_golden(dgs, seed):
    gold = read_sections(os.path.join(HERE, "golden", "lowrank16384_parallel.txt"))[f"seed{seed}"]
    say(f"parallel case lowrank16384 seed {seed}")
    A = gen.lowrank_matrix(16384, seed)
    tau, res = dgs.solve(A, parallel=True)
    h = hashlib.sha256(np.ascontiguousarray(tau, dtype="<i4").tobytes()).hexdigest()
    assert res["initial_benefit"] == int(gold["greedy_f"])
    assert res["total_benefit"] == int(gold["f"])
    assert res["switches"] == int(gold["S"]) and res["rounds"] == int(gold["rounds"])
    assert h == gold["tau_sha256"]


def test_ordered_walk_above_16384(dgs):
    # n > 16384 takes the single-wave ordered walk of Check Conflicts instead
    # of the in-LDS iteration; its first rounds must give the oracle's result
    # (ties: benefits from a small range)
    check(dgs, gen.uniform_matrix(16400, 0, 1000, 5), max_rounds=2, what="uniform n=16400, two rounds")


def test_lowrank20480_golden(dgs):
    """The complete run above 16384 (walking Check Conflicts) against the
    oracle's, stored by make_golden.py --full20480."""
    gold = read_sections(os.path.join(HERE, "golden", "lowrank20480.txt"))["parallel_seed1"]
    n = int(gold["n"])
    say(f"parallel case lowrank{n} seed 1")
    A = gen.lowrank_matrix(n, 1)
    tau, res = dgs.solve(A, parallel=True)
    h = hashlib.sha256(np.ascontiguousarray(tau, dtype="<i4").tobytes()).hexdigest()
    assert res["initial_benefit"] == int(gold["greedy_f"])
    assert res["total_benefit"] == int(gold["f"])
    assert res["switches"] == int(gold["S"]) and res["rounds"] == int(gold["rounds"])
    assert h == gold["tau_sha256"]
