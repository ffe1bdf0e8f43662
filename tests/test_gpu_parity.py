"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Integer work, so the bar is bit-exact: the same assignment permutation,
the same total benefit and the same number of switches.  Inputs come from
workloads.gen (seeded); expected values from the oracle (live) or, at
n = 16384 where the oracle needs minutes, from tests/golden/lowrank16384.txt
written by tests/golden/make_golden.py (oracle only).
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np
import pytest

import oracle
from tests.golden_io import ints, matrix, read_sections, worked_examples
from workloads import gen

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dgs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1106_5694_amd as m
    m.lib()
    return m


def check_against_oracle(dgs, A, init=None, max_switches=-1, what=""):
    say(f"case {what}: n={A.shape[0]} init={'yes' if init is not None else 'greedy'} k={max_switches}")
    tau, res = dgs.solve(A, init=init, max_switches=max_switches)
    ref = oracle.dgs_incr(A, init=init, max_switches=max_switches)
    assert oracle.is_permutation(tau)
    assert (tau == ref["tau"]).all(), what
    assert res["total_benefit"] == ref["f"], what
    assert res["switches"] == ref["S"], what
    assert res["total_benefit"] == oracle.objective(A, tau)
    return tau, res


@pytest.mark.parametrize("name", sorted(worked_examples()))
def test_worked_examples(dgs, name):
    ex = worked_examples()[name]
    A = matrix(ex["A"])
    tau, res = dgs.solve(A)
    assert list(tau) == ints(ex["tau"])
    assert res["total_benefit"] == int(ex["f"]) and res["switches"] == int(ex["S"])
    assert res["initial_benefit"] == int(ex["greedy_f"])
    tau0, _ = dgs.solve(A, max_switches=0)
    assert list(tau0) == ints(ex["greedy"])
    g, j = dgs.diff_eval(A, np.array(ints(ex["greedy"]), dtype=np.int32))
    if "scan0_gain" in ex:
        assert list(g) == ints(ex["scan0_gain"]) and list(j) == ints(ex["scan0_job"])
    else:
        assert g[0] == np.iinfo(np.int64).min and j[0] == -1


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_uniform256(dgs, seed):
    check_against_oracle(dgs, gen.single_instance("uniform256", seed), what=f"uniform256 seed {seed}")


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 127, 255, 257, 1000])
@pytest.mark.parametrize("kind", ["ties", "signed", "lowrank"])
def test_edge_sizes(dgs, n, kind):
    if kind == "ties":
        A = gen.uniform_matrix(n, 0, 3, 100 + n)
    elif kind == "signed":
        A = gen.uniform_matrix(n, -1000, 1000, 200 + n)
    else:
        A = gen.lowrank_matrix(n, 300 + n)
    check_against_oracle(dgs, A, what=f"edge {kind} n={n}")


def test_extreme_values(dgs):
    m = (1 << 29) - 1
    A = gen.uniform_matrix(300, -m, m + 1, 9)
    A[0, 0], A[1, 1], A[2, 5] = m, -m, m
    check_against_oracle(dgs, A, what="extreme values")


def test_out_of_range_rejected(dgs):
    A = gen.uniform_matrix(64, 0, 100, 1)
    A[3, 7] = 1 << 29
    with pytest.raises(dgs.DGSError) as e:
        dgs.solve(A)
    assert e.value.status == dgs.DGS_E_RANGE
    A[3, 7] = -(1 << 29)
    with pytest.raises(dgs.DGSError) as e:
        dgs.solve(A)
    assert e.value.status == dgs.DGS_E_RANGE


def test_bad_init_rejected(dgs):
    A = gen.uniform_matrix(32, 0, 100, 1)
    bad = np.arange(32, dtype=np.int32)
    bad[5] = 6
    with pytest.raises(dgs.DGSError) as e:
        dgs.solve(A, init=bad)
    assert e.value.status == dgs.DGS_E_INVAL


@pytest.mark.parametrize("n,seed", [(256, 1), (777, 2)])
def test_random_start(dgs, n, seed):
    # the paper's random start (Section 3.1) through init_assign
    A = gen.lowrank_matrix(n, seed)
    check_against_oracle(dgs, A, init=gen.permutation(n, seed), what="random start")


def test_anytime_prefix_and_resume(dgs):
    A = gen.lowrank_matrix(500, 4)
    full = oracle.dgs_incr(A)
    assert full["S"] > 20
    for k in (0, 1, 7, full["S"] // 2, full["S"], full["S"] + 5):
        tau_k, res_k = check_against_oracle(dgs, A, max_switches=k, what=f"prefix {k}")
        tau_r, res_r = dgs.solve(A, init=tau_k)
        assert (tau_r == full["tau"]).all() and res_r["total_benefit"] == full["f"]
        assert res_r["switches"] == full["S"] - min(k, full["S"])


@pytest.mark.parametrize("n,kind", [(256, "greedy"), (256, "random"), (1000, "random"), (4096, "greedy")])
def test_diff_eval(dgs, n, kind):
    A = gen.uniform_matrix(n, 0, 1000, 5) if n < 4096 else gen.lowrank_matrix(n, 5)
    tau = oracle.greedy(A) if kind == "greedy" else gen.permutation(n, 3)
    say(f"case diff_eval n={n} {kind}")
    g, j = dgs.diff_eval(A, tau)
    rg, rj = oracle.scan(A, tau)
    assert (g == rg).all() and (j == rj).all()


def test_device_pointers(dgs):
    import torch
    A = gen.lowrank_matrix(700, 8)
    ref = oracle.dgs_incr(A)
    Ad = torch.from_numpy(A).cuda()
    tau, res = dgs.solve(Ad)
    torch.cuda.synchronize()
    assert tau.is_cuda and (tau.cpu().numpy() == ref["tau"]).all()
    assert res["total_benefit"] == ref["f"] and res["switches"] == ref["S"]
    g, j = dgs.diff_eval(Ad, torch.from_numpy(ref["tau"]).cuda())
    rg, rj = oracle.scan(A, ref["tau"])
    assert (g.cpu().numpy() == rg).all() and (j.cpu().numpy() == rj).all()


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_lowrank4096(dgs, seed):
    check_against_oracle(dgs, gen.single_instance("lowrank4096", seed), what=f"lowrank4096 seed {seed}")


def _golden16384():
    path = os.path.join(os.path.dirname(__file__), "golden", "lowrank16384.txt")
    return read_sections("lowrank16384.txt") if os.path.exists(path) else {}


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_lowrank16384(dgs, seed):
    gold = _golden16384().get(f"seed{seed}")
    if gold is None:
        pytest.skip("golden values for this seed not generated")
    say(f"case lowrank16384 seed {seed}")
    A = gen.single_instance("lowrank16384", seed)
    tau, res = dgs.solve(A)
    assert res["initial_benefit"] == int(gold["greedy_f"])
    assert res["total_benefit"] == int(gold["f"]) and res["switches"] == int(gold["S"])
    h = hashlib.sha256(np.ascontiguousarray(tau, dtype="<i4").tobytes()).hexdigest()
    assert h == gold["tau_sha256"]
    # properties that hold at any size, on sampled agents: a permutation, and
    # no improving 2-exchange left for them (every gain by its definition)
    assert oracle.is_permutation(tau)
    rows = gen.permutation(16384, seed)[:64]
    d = A[np.arange(16384), tau].astype(np.int64)
    for i in rows:
        g = (A[i, tau].astype(np.int64) + A[:, tau[i]].astype(np.int64)) - (d[i] + d)
        assert g.max() <= 0


def test_lowrank20480_wide_gather(dgs):
    """n = 20480 takes 80 switching workgroups, the kernel variant that
    gathers more than 8 exchange words per thread.  Its first 1000 switches
    (make_golden.py --prefix) and its complete run (make_golden.py
    --full20480) match the oracle's."""
    gold = read_sections("lowrank20480_prefix.txt")["seed1"]
    n, k = int(gold["n"]), int(gold["k"])
    say(f"case lowrank{n} seed 1 prefix k={k} and full run")
    A = gen.lowrank_matrix(n, 1)
    tau, res = dgs.solve(A, max_switches=k)
    assert res["initial_benefit"] == int(gold["greedy_f"])
    assert res["total_benefit"] == int(gold["f"]) and res["switches"] == int(gold["S"])
    h = hashlib.sha256(np.ascontiguousarray(tau, dtype="<i4").tobytes()).hexdigest()
    assert h == gold["tau_sha256"]
    full = read_sections("lowrank20480.txt")["steepest_seed1"]
    assert int(full["n"]) == n
    tau2, res2 = dgs.solve(A)
    assert res2["initial_benefit"] == int(full["greedy_f"])
    assert res2["total_benefit"] == int(full["f"]) and res2["switches"] == int(full["S"])
    h2 = hashlib.sha256(np.ascontiguousarray(tau2, dtype="<i4").tobytes()).hexdigest()
    assert h2 == full["tau_sha256"]


def test_ragged_large_prefix(dgs):
    """n = 16387: rows that are not a multiple of four and longer than one
    LDS chunk when the switching loop's permuted copy of A is built; the first
    300 switches from the greedy start match the oracle's."""
    A = gen.lowrank_matrix(16387, 5)
    check_against_oracle(dgs, A, max_switches=300, what="ragged large prefix")


def test_plain_dgs_solve(dgs):
    """The three-argument dgs_solve, called through ctypes with host buffers."""
    import ctypes
    A = gen.lowrank_matrix(300, 21)
    out = np.full(300, -7, dtype=np.int32)
    st = dgs.lib().dgs_solve(A.ctypes.data, 300, out.ctypes.data)
    assert st == dgs.DGS_OK
    ref = oracle.dgs_incr(A)
    assert (out == ref["tau"]).all()
    # an error leaves the output untouched
    bad = np.full(300, -7, dtype=np.int32)
    assert dgs.lib().dgs_solve(ctypes.c_void_p(0), 300, bad.ctypes.data) == dgs.DGS_E_INVAL
    assert (bad == -7).all()


def test_size_limits(dgs):
    """n above the steepest-ascent limit is refused before any buffer is read
    (a one-entry buffer stands in for the matrix), as is n above DGS_MAX_N."""
    import ctypes
    one = np.zeros(1, dtype=np.int32)
    out = np.zeros(1, dtype=np.int32)
    L = dgs.lib()
    assert L.dgs_solve(one.ctypes.data, 65536, out.ctypes.data) == dgs.DGS_E_INVAL
    assert b"65535" in L.dgs_last_error()
    assert L.dgs_solve(one.ctypes.data, 262145, out.ctypes.data) == dgs.DGS_E_INVAL
    lazy = dgs.Options(-1, None, dgs.DGS_LAZY, None)
    assert L.dgs_solve_ex(one.ctypes.data, 16385, out.ctypes.data, ctypes.byref(lazy), None) == dgs.DGS_E_INVAL


def test_batched_equals_solo(dgs):
    ns = [64, 1, 2, 300, 1000, 65, 777]
    As = [gen.uniform_matrix(n, 0, 10000, 40 + i) for i, n in enumerate(ns)]
    say("case batched")
    taus, results = dgs.solve_batched(As)
    for A, tau, res in zip(As, taus, results):
        ref = oracle.dgs_incr(A)
        assert (tau == ref["tau"]).all()
        assert res["total_benefit"] == ref["f"] and res["switches"] == ref["S"]


def test_server_equals_solo(dgs):
    # small requests (batched launches) and large ones (concurrent switching
    # loops on worker streams) in one mix: each result equals the same
    # instance solved alone, and the oracle
    ns = [128, 2500, 300, 64, 3000, 1000, 257, 2049, 5, 2300]
    As = [gen.lowrank_matrix(n, 60 + i) for i, n in enumerate(ns)]
    say(f"case server mix: {ns}")
    with dgs.Server(max_slots=6) as srv:
        tickets = [srv.submit(A) for A in As]
        outs = [srv.wait(t, timeout_us=120_000_000) for t in tickets]
        st = srv.stats()
    for A, out in zip(As, outs):
        assert out is not None
        alone, res_alone = dgs.solve(A)
        assert (out[0] == alone).all() and out[1]["total_benefit"] == res_alone["total_benefit"]
        assert out[1]["switches"] == res_alone["switches"]
        ref = oracle.dgs_incr(A)
        assert (out[0] == ref["tau"]).all() and out[1]["total_benefit"] == ref["f"]
    assert st["completed"] == len(As) and st["queued"] == 0
    assert 0 < st["p50_us"] <= st["p99_us"]


def test_server_poll(dgs):
    """dgs_server_poll: DGS_E_AGAIN while pending, then the result once."""
    A = gen.lowrank_matrix(3000, 31)
    ref = oracle.dgs_incr(A)
    say("case server poll n=3000")
    with dgs.Server() as srv:
        t = srv.submit(A)
        out, polls = None, 0
        deadline = __import__("time").time() + 120
        while out is None:
            out = srv.poll(t)
            polls += 1
            assert __import__("time").time() < deadline
        assert (out[0] == ref["tau"]).all() and out[1]["total_benefit"] == ref["f"]
        with pytest.raises(dgs.DGSError) as e:  # the ticket was consumed
            srv.poll(t)
        assert e.value.status == dgs.DGS_E_INVAL
    say(f"server poll: {polls} polls")


def test_server_budget_admission(dgs):
    # a budget that holds one large request at a time still completes every
    # request; a request that can never fit is refused at submit
    n = 2200
    budget = dgs.server_footprint(n) + dgs.server_footprint(512)
    As = [gen.uniform_matrix(n, 0, 1000, 80 + i) for i in range(3)] + [gen.uniform_matrix(512, 0, 1000, 90)]
    with dgs.Server(hbm_budget_bytes=budget) as srv:
        tickets = [srv.submit(A) for A in As]
        outs = [srv.wait(t, timeout_us=120_000_000) for t in tickets]
        with pytest.raises(dgs.DGSError) as e:
            srv.submit(gen.uniform_matrix(3000, 0, 10, 1))
        assert e.value.status == dgs.DGS_E_NOMEM
    for A, out in zip(As, outs):
        ref = oracle.dgs_incr(A)
        assert (out[0] == ref["tau"]).all() and out[1]["switches"] == ref["S"]


def test_server_memory_within_budget(dgs):
    """Device memory the server holds (hipMemGetInfo, sampled while requests of
    mixed sizes run and after they finish) stays within its budget plus a
    small allowance for the pool's granularity, and every result is the
    oracle's."""
    import time

    import torch
    MiB = 1 << 20
    budget = dgs.server_footprint(3000) + dgs.server_footprint(1500)
    ns = [2100, 2600, 3000, 2300, 500, 1500, 2800, 100, 2900, 2200, 1800]
    As = [gen.lowrank_matrix(n, 500 + i) for i, n in enumerate(ns)]
    say(f"case server memory budget {budget / MiB:.0f} MiB: {ns}")
    torch.cuda.synchronize()
    with dgs.Server(hbm_budget_bytes=budget) as srv:
        srv.wait(srv.submit(As[7]), timeout_us=60_000_000)  # workers and their streams are up
        time.sleep(0.2)
        free0 = torch.cuda.mem_get_info()[0]
        tickets = [srv.submit(A) for A in As]
        outs, lowest = [None] * len(As), free0
        deadline = time.time() + 300
        while any(o is None for o in outs):
            for k, t in enumerate(tickets):
                if outs[k] is None:
                    outs[k] = srv.poll(t)
            lowest = min(lowest, torch.cuda.mem_get_info()[0])
            assert time.time() < deadline
        held_after = free0 - torch.cuda.mem_get_info()[0]
    held_peak = free0 - lowest
    say(f"server memory: peak {held_peak / MiB:.0f} MiB, after {held_after / MiB:.0f} MiB, "
        f"budget {budget / MiB:.0f} MiB")
    assert held_peak <= budget + 64 * MiB
    assert held_after <= budget + 64 * MiB
    for A, out in zip(As, outs):
        ref = oracle.dgs_incr(A)
        assert (out[0] == ref["tau"]).all() and out[1]["total_benefit"] == ref["f"]


def test_batched_workload_sample(dgs):
    # the batched workload's shape: log-uniform n in [64, 2048], benefits in [0, 10000);
    # every instance of a mixed batch equals the oracle, and one instance above the
    # single-workgroup limit takes the single-instance path inside the same call
    ns = list(gen.loguniform_sizes(48, 64, 2048, 7)) + [2048, 2049, 3000]
    As = [gen.uniform_matrix(int(n), 0, 10000, 900 + i) for i, n in enumerate(ns)]
    say(f"case batched sample: {len(As)} instances, max n {max(ns)}")
    taus, results = dgs.solve_batched(As)
    for A, tau, res in zip(As, taus, results):
        ref = oracle.dgs_incr(A)
        assert (tau == ref["tau"]).all()
        assert res["total_benefit"] == ref["f"] and res["switches"] == ref["S"]
        assert res["initial_benefit"] == oracle.objective(A, oracle.greedy(A))


def test_batched_device_pointers_and_prefix(dgs):
    import torch
    ns = [5, 130, 700, 1500]
    As = [gen.lowrank_matrix(n, 70 + i) for i, n in enumerate(ns)]
    Ads = [torch.from_numpy(A).cuda() for A in As]
    taus, results = dgs.solve_batched(Ads, max_switches=3)
    torch.cuda.synchronize()
    for A, tau, res in zip(As, taus, results):
        ref = oracle.dgs_incr(A, max_switches=3)
        assert (tau.cpu().numpy() == ref["tau"]).all() and res["switches"] == ref["S"]


def test_batched_out_of_range(dgs):
    As = [gen.uniform_matrix(100, 0, 10, 1), gen.uniform_matrix(50, 0, 10, 2)]
    As[1][3, 4] = -(1 << 29)
    with pytest.raises(dgs.DGSError) as e:
        dgs.solve_batched(As)
    assert e.value.status == dgs.DGS_E_RANGE
