"""GPU: batch plans (graph-captured persistent launch, autotuned workgroup
size) against the CPU oracle.  Integer results: bit-exact per instance."""
from __future__ import annotations

import math
import os
import sys

import numpy as np
import pytest

import oracle
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


def _refs(As, max_switches=-1):
    return [oracle.dgs_incr(A, max_switches=max_switches) for A in As]


def _check(taus, results, refs):
    for tau, res, ref in zip(taus, results, refs):
        assert (tau == ref["tau"]).all()
        assert res["total_benefit"] == ref["f"] and res["switches"] == ref["S"]


def size_class(ns):
    # the plan's size class: count, largest n rounded up to a power of two,
    # floor(log2(total entries))
    p2 = 1
    while p2 < max(ns):
        p2 <<= 1
    entries = sum(n * n for n in ns)
    return f"c{len(ns)}_n{p2}_e{entries.bit_length() - 1}"


def test_plan_graph_replays(dgs):
    # several replays of one captured graph, with new inputs, resident inputs
    # and eager library work in between; every replay is checked
    ns = [int(n) for n in gen.loguniform_sizes(20, 64, 2048, 11)] + [2048, 1, 2]
    X = [gen.uniform_matrix(n, 0, 10000, 500 + i) for i, n in enumerate(ns)]
    Y = [gen.uniform_matrix(n, 0, 10000, 700 + i) for i, n in enumerate(ns)]
    rx, ry = _refs(X), _refs(Y)
    say(f"case plan replays: {len(ns)} instances, max n {max(ns)}")
    with dgs.BatchPlan(ns, autotune=True) as plan:
        taus, res = plan.run(X)
        _check(taus, res, rx)
        assert plan.config()[0] in (256, 512)
        taus, res = plan.run(Y)
        _check(taus, res, ry)
        dgs.solve(X[0])  # eager work between replays
        taus, res = plan.run(None)  # Y is still resident
        _check(taus, res, ry)
        taus, res = plan.run(X)
        _check(taus, res, rx)
        _, res = plan.run(None, outs=False)
        assert [r["total_benefit"] for r in res] == [r["f"] for r in rx]


@pytest.mark.parametrize("block", [256, 512])
def test_plan_forced_block(dgs, tmp_path, monkeypatch, block):
    # a tuning-cache entry fixes the workgroup size; results do not depend on it
    ns = [int(n) for n in gen.loguniform_sizes(12, 64, 1500, 13 + block)]
    As = [gen.lowrank_matrix(n, 40 + i) for i, n in enumerate(ns)]
    cache = tmp_path / f"tune{block}.txt"
    cache.write_text(f"{size_class(ns)} {block}\n")
    monkeypatch.setenv("DGS_TUNE_CACHE", str(cache))
    with dgs.BatchPlan(ns, max_switches=7) as plan:
        assert plan.config()[0] == block
        taus, res = plan.run(As)
    _check(taus, res, _refs(As, max_switches=7))


def test_plan_autotune_writes_cache(dgs, tmp_path, monkeypatch):
    ns = [300, 77, 1024, 5]
    As = [gen.uniform_matrix(n, 0, 100, 60 + i) for i, n in enumerate(ns)]
    cache = tmp_path / "tune.txt"
    cache.write_text("")
    monkeypatch.setenv("DGS_TUNE_CACHE", str(cache))
    with dgs.BatchPlan(ns, autotune=True) as plan:
        taus, res = plan.run(As)
        block = plan.config()[0]
    _check(taus, res, _refs(As))
    lines = cache.read_text().split()
    assert lines[-2:] == [size_class(ns), str(block)]


def test_plan_rejects(dgs):
    with pytest.raises(dgs.DGSError) as e:
        dgs.BatchPlan([100, 2049])
    assert e.value.status == dgs.DGS_E_INVAL
    As = [gen.uniform_matrix(64, 0, 10, 1), gen.uniform_matrix(80, 0, 10, 2)]
    As[1][5, 6] = 1 << 29
    with dgs.BatchPlan([64, 80]) as plan:
        with pytest.raises(dgs.DGSError) as e:
            plan.run(As)
        assert e.value.status == dgs.DGS_E_RANGE
        As[1][5, 6] = 3
        taus, res = plan.run(As)
        _check(taus, res, _refs(As))
