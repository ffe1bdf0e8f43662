"""GPU parity of rectangular DGS (n agents, m >= n jobs; dgs_solve_rect)
against oracle.rect_dgs / rect_dgs_full, which work on the rectangle
directly (swaps and moves to unassigned jobs), bit-exact: assignment, total
benefit, switches.  The library runs the m - n unassigned jobs as virtual
agents of benefit 0 whose rows are never stored, so this also checks that
reduction; from both starts (agent-order and global greedy)."""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu

RECT_A = np.array([[3, 1, 0], [9, 0, 4]], dtype=np.int32)  # worked by hand in tests/test_oracle.py


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
    say(f"rect case {what}: {A.shape[0]} x {A.shape[1]} init={'yes' if init is not None else 'greedy'}")
    tau, res = dgs.solve_rect(A, init=init, max_switches=max_switches)
    ref = oracle.rect_dgs(A, init=init, max_switches=max_switches)
    assert len(set(tau.tolist())) == A.shape[0] and tau.min() >= 0 and tau.max() < A.shape[1]
    assert (tau == ref["tau"]).all(), what
    assert res["total_benefit"] == ref["f"] == int(A[np.arange(A.shape[0]), tau].sum()), what
    assert res["switches"] == ref["S"], what
    return tau, res


def test_worked_example(dgs):
    tau, res = dgs.solve_rect(RECT_A)
    assert list(tau) == [1, 0] and res["total_benefit"] == 10 and res["switches"] == 2
    assert res["initial_benefit"] == 7


@pytest.mark.parametrize("n,m", [(1, 1), (1, 5), (3, 7), (64, 65), (100, 300), (257, 400), (500, 512), (300, 1000)])
@pytest.mark.parametrize("kind", ["uniform", "lowrank", "ties"])
def test_shapes(dgs, n, m, kind):
    if kind == "uniform":
        A = gen.uniform_matrix(m, -500, 1000, n + m)[:n]
    elif kind == "lowrank":
        A = gen.lowrank_matrix(m, n + 2 * m)[:n]
    else:
        A = gen.uniform_matrix(m, 0, 3, n + 3 * m)[:n]
    check(dgs, np.ascontiguousarray(A), what=f"{kind}")


def test_square_equals_solve(dgs):
    A = gen.lowrank_matrix(700, 8)
    t1, r1 = dgs.solve_rect(A)
    t2, r2 = dgs.solve(A)
    assert (t1 == t2).all() and r1["total_benefit"] == r2["total_benefit"] and r1["switches"] == r2["switches"]


def test_start_prefix_and_device(dgs):
    import torch
    A = np.ascontiguousarray(gen.lowrank_matrix(600, 21)[:400])
    init = gen.permutation(600, 21)[:400].astype(np.int32)
    check(dgs, A, init=init, what="given start")
    for k in (0, 1, 25):
        check(dgs, A, max_switches=k, what=f"prefix {k}")
    tau, res = dgs.solve_rect(torch.from_numpy(A).cuda(), init=torch.from_numpy(init).cuda())
    ref = oracle.rect_dgs(A, init=init)
    assert (tau.cpu().numpy() == ref["tau"]).all() and res["total_benefit"] == ref["f"]


def test_rejected_calls(dgs):
    L = dgs.lib()
    A = np.ascontiguousarray(gen.uniform_matrix(8, 0, 9, 1)[:5])
    out = np.empty(8, dtype=np.int32)
    res = dgs.Result()

    def call(n, m, flags=0, init=None):
        opt = dgs.Options(max_switches=-1, init_assign=None if init is None else init.ctypes.data,
                          flags=flags, stream=None)
        return L.dgs_solve_rect(A.ctypes.data, n, m, out.ctypes.data, ctypes.byref(opt), ctypes.byref(res))

    assert call(6, 5) == dgs.DGS_E_INVAL          # n > m
    assert call(5, 8, flags=dgs.DGS_PARALLEL) == dgs.DGS_E_INVAL
    assert call(5, 8, flags=dgs.DGS_LAZY) == dgs.DGS_E_INVAL
    assert call(5, 8, init=np.array([0, 1, 2, 3, 3], dtype=np.int32)) == dgs.DGS_E_INVAL
    assert call(5, 8, init=np.array([0, 1, 2, 3, 8], dtype=np.int32)) == dgs.DGS_E_INVAL
    assert call(5, 8) == dgs.DGS_OK
    assert list(out[:5]) == list(oracle.rect_dgs(A)["tau"])


# ---- without an m x m buffer; the global greedy start ------------------------------------


@pytest.mark.parametrize("n,m", [(1, 5000), (3, 64), (63, 64), (130, 1000), (257, 2050), (1001, 1003)])
def test_virtual_agents_edge_shapes(dgs, n, m):
    A = np.ascontiguousarray(gen.uniform_matrix(m, -300, 300, 5 * n + m)[:n])
    check(dgs, A, what="edge")


@pytest.mark.parametrize("n,m", [(1, 1), (2, 9), (40, 40), (100, 300), (257, 400), (500, 512), (300, 1000)])
@pytest.mark.parametrize("kind", ["uniform", "lowrank", "ties"])
def test_global_greedy_start_and_solve(dgs, n, m, kind):
    """The device's global greedy start (max_switches = 0) equals the oracle's
    sorted walk, and the solve from it equals the oracle's rectangular DGS
    from that start."""
    if kind == "uniform":
        A = gen.uniform_matrix(m, -500, 1000, 7 * n + m)[:n]
    elif kind == "lowrank":
        A = gen.lowrank_matrix(m, 7 * n + 2 * m, rows=n)
    else:
        A = gen.uniform_matrix(m, 0, 3, 7 * n + 3 * m)[:n]
    A = np.ascontiguousarray(A)
    say(f"global greedy case {kind}: {n} x {m}")
    gg = oracle.global_greedy(A)
    tau0, res0 = dgs.solve_rect(A, max_switches=0, global_greedy=True)
    assert (tau0 == gg).all() and res0["switches"] == 0
    assert res0["initial_benefit"] == int(A[np.arange(n), gg].sum())
    tau, res = dgs.solve_rect(A, global_greedy=True)
    ref = oracle.rect_dgs_full(A, init=gg)
    assert (tau == ref["tau"]).all() and res["total_benefit"] == ref["f"] and res["switches"] == ref["S"]


def test_global_greedy_square_solve(dgs):
    """dgs_solve_ex with the global greedy start on square instances."""
    for n, seed in ((100, 1), (1000, 2)):
        A = gen.lowrank_matrix(n, 40 + seed)
        gg = oracle.global_greedy(A)
        tau, res = dgs.solve(A, global_greedy=True)
        ref = oracle.dgs_incr(A, init=gg)
        assert (tau == ref["tau"]).all() and res["total_benefit"] == ref["f"] and res["switches"] == ref["S"]
        assert res["initial_benefit"] == oracle.objective(A, gg)


def _golden_rect():
    from tests.golden_io import read_sections
    return read_sections("rect1000x16384.txt")


def _sha(t):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(t, dtype="<i4").tobytes()).hexdigest()


def test_rect_1000x16384_against_golden(dgs):
    """1000 agents, 16384 jobs (the first 1000 rows of the n = 16384 low-rank
    workload): both starts, bit-exact with the oracle's stored results, and
    the library's device memory for the solve stays far below one m x m
    matrix (4 m^2 = 1 GiB)."""
    import torch
    g = _golden_rect()
    A = gen.lowrank_matrix(16384, 1, rows=1000)
    Ad = torch.from_numpy(A).cuda()
    torch.cuda.synchronize()
    dgs.release_cached()
    free0, _ = torch.cuda.mem_get_info()
    for sec, gg in (("greedy_seed1", False), ("global_seed1", True)):
        say(f"rect 1000 x 16384, {sec}")
        exp = g[sec]
        tau0, r0 = dgs.solve_rect(Ad, max_switches=0, global_greedy=gg)
        assert r0["initial_benefit"] == int(exp["start_f"])
        if gg:
            assert _sha(tau0.cpu().numpy()) == exp["start_sha256"]
        tau, res = dgs.solve_rect(Ad, global_greedy=gg)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        t = tau.cpu().numpy()
        assert len(set(t.tolist())) == 1000 and t.min() >= 0 and t.max() < 16384
        assert res["total_benefit"] == int(exp["f"]) == int(A[np.arange(1000), t].sum())
        assert res["switches"] == int(exp["S"])
        assert _sha(t) == exp["tau_sha256"]
        assert free0 - free1 < 256 << 20, (free0, free1)  # AT (64 MiB) + vectors, no 1 GiB matrix
