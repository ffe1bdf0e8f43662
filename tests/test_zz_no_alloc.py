"""dgs_solve_noalloc (the entry point for callers that cannot allocate)
against dgs_solve_ex on the same device-resident instances, through the C
ABI: two calls in a row, the second on a smaller instance, each bit-exact
(assignment, objective, switch count) with the allocating entry point."""
import ctypes

import numpy as np
import pytest

import paper_1106_5694_amd as dgs
from workloads import gen

pytestmark = pytest.mark.gpu


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _noalloc(torch, A, init=None, max_switches=-1):
    n = A.shape[0]
    out = torch.full((n,), -7, dtype=torch.int32, device="cuda:0")
    res = dgs.solve_noalloc(A, out, init=init, max_switches=max_switches)
    torch.cuda.synchronize()
    return out.cpu().numpy(), res


def _alloc(torch, A, init=None, max_switches=-1):
    tau, res = dgs.solve(A, init=init, max_switches=max_switches)
    torch.cuda.synchronize()
    return tau.cpu().numpy(), res


def _same(a, b):
    (ta, ra), (tb, rb) = a, b
    assert np.array_equal(ta, tb)
    for k in ("initial_benefit", "total_benefit", "switches", "rescans", "stalls"):
        assert ra[k] == rb[k], k


@pytest.mark.parametrize("sizes", [(4096, 1000), (3000, 257)])
def test_noalloc_matches_solve_ex_twice(sizes):
    torch = _torch()
    for n, seed in zip(sizes, (1, 2)):
        print(f"noalloc: n={n} seed={seed}", flush=True)
        A = (gen.lowrank_matrix(n, seed) if n >= 1000 else gen.uniform_matrix(n, 0, 1000, seed))
        Ad = torch.from_numpy(A).to("cuda:0")
        _same(_noalloc(torch, Ad), _alloc(torch, Ad))


def test_noalloc_start_prefix_and_tiny():
    torch = _torch()
    A = torch.from_numpy(gen.uniform_matrix(512, 0, 50, 3)).to("cuda:0")
    init = torch.from_numpy(np.random.default_rng(3).permutation(512).astype(np.int32)).to("cuda:0")
    _same(_noalloc(torch, A, init=init), _alloc(torch, A, init=init))
    _same(_noalloc(torch, A, max_switches=17), _alloc(torch, A, max_switches=17))
    for n in (1, 2, 65):
        B = torch.from_numpy(gen.uniform_matrix(n, -20, 20, n)).to("cuda:0")
        _same(_noalloc(torch, B), _alloc(torch, B))


def test_noalloc_allocates_nothing():
    torch = _torch()
    A = torch.from_numpy(gen.lowrank_matrix(2048, 4)).to("cuda:0")
    out = torch.empty(2048, dtype=torch.int32, device="cuda:0")
    dgs.solve_noalloc(A, out)  # set-up happened before: the first call on the device
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    B = A[:1024, :1024].contiguous()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    for M in (A, B, A):
        dgs.solve_noalloc(M, out[:M.shape[0]])
    torch.cuda.synchronize()
    free2, _ = torch.cuda.mem_get_info()
    assert free2 == free1, (free0, free1, free2)


def test_noalloc_rejects():
    torch = _torch()
    L = dgs.lib()
    big = torch.zeros((dgs.NOALLOC_MAX_N + 1, dgs.NOALLOC_MAX_N + 1), dtype=torch.int32, device="cuda:0")
    out = torch.empty(dgs.NOALLOC_MAX_N + 1, dtype=torch.int32, device="cuda:0")
    assert L.dgs_solve_noalloc(big.data_ptr(), dgs.NOALLOC_MAX_N + 1, out.data_ptr(), None, None) == dgs.DGS_E_INVAL
    A = torch.from_numpy(gen.uniform_matrix(64, 0, 100, 5)).to("cuda:0")
    bad = torch.zeros(64, dtype=torch.int32, device="cuda:0")  # not a permutation
    opt = dgs.Options(max_switches=-1, init_assign=bad.data_ptr(), flags=dgs.DGS_DEVICE_PTRS, stream=None)
    assert L.dgs_solve_noalloc(A.data_ptr(), 64, out.data_ptr(), ctypes.byref(opt), None) == dgs.DGS_E_INVAL
    opt = dgs.Options(max_switches=-1, init_assign=None, flags=dgs.DGS_DEVICE_PTRS | dgs.DGS_PARALLEL, stream=None)
    assert L.dgs_solve_noalloc(A.data_ptr(), 64, out.data_ptr(), ctypes.byref(opt), None) == dgs.DGS_E_INVAL
    with pytest.raises(dgs.DGSError):
        A2 = A.clone()
        A2[3, 3] = (1 << 29)
        dgs.solve_noalloc(A2, out[:64])
