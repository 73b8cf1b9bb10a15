"""GPU test of ufem_cg_iterate_static, the CG entry point that allocates
nothing (its workspace is a fixed device array of the library): the same
iterations as ufem_cg_iterate with a caller-provided workspace, on two calls
in a row, the second on a smaller problem, in both precisions; sizes beyond
the fixed workspace are rejected."""
import ctypes as C
import sys

import numpy as np
import pytest

import ufem_inputs as ui

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ops(torch, wl, seed_vec):
    from paper_2404_07911_amd import Operator, Plan, Problem

    op = Operator(Plan(Problem.from_workload(wl)))
    rng = np.random.default_rng(seed_vec)
    b = torch.from_numpy(rng.uniform(-1, 1, op.n_dofs)).cuda()
    return op, b


def _run_both(torch, op, b, dtype, n_iter):
    from paper_2404_07911_amd import _lib as L

    prec = L.F64 if dtype == torch.float64 else L.F32
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    vp = lambda t: C.c_void_p(t.data_ptr())
    r0 = b.to(dtype)
    # reference: ufem_cg_iterate with a caller-provided workspace
    x1 = torch.zeros_like(r0)
    r1 = r0.clone()
    p1 = r0.clone()
    ap = torch.empty_like(r0)
    scal = torch.zeros(4, dtype=torch.float64, device="cuda")
    L.check(L.lib().ufem_dot(prec, op.n_dofs, vp(r1), vp(r1), vp(scal), s))
    L.check(L.lib().ufem_cg_iterate(op._h, prec, n_iter, vp(x1), vp(r1), vp(p1), vp(ap), vp(scal), s))
    # the entry point without workspace
    x2 = torch.zeros_like(r0)
    r2 = r0.clone()
    p2 = r0.clone()
    res = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    L.check(L.lib().ufem_cg_iterate_static(op._h, prec, n_iter, vp(x2), vp(r2), vp(p2), vp(res), s))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return (x1, r1, p1, scal.cpu().numpy()), (x2, r2, p2, res.cpu().numpy()), free0 - free1


def _rel(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_static_cg_matches_workspace_cg(torch, dtype_name):
    dtype = getattr(torch, dtype_name)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    big, bb = _ops(torch, ui.ball3d(5, n=10, degree=2)[0], 1)
    small, bs = _ops(torch, ui.disk2d(0)[0], 2)
    assert small.n_dofs < big.n_dofs
    for name, op, b in (("ball p2 10^3", big, bb), ("disk p2 16^2", small, bs)):
        _say(f"[static cg] {name} {dtype_name}")
        ref, got, dmem = _run_both(torch, op, b, dtype, 9)
        for i in range(3):
            assert _rel(got[i], ref[i]) < tol, (name, i)
        assert abs(got[3][0] - ref[3][0]) <= tol * abs(ref[3][0])
        assert got[3][1] == ref[3][3] == 0.0
        assert dmem == 0, dmem


def test_static_cg_rejects_sizes_beyond_the_workspace(torch):
    from paper_2404_07911_amd import Operator, Plan, Problem, UfemError
    from paper_2404_07911_amd import _lib as L

    wl, _ = ui.ball3d(0, n=64, degree=4)
    op = Operator(Plan(Problem.from_workload(wl)))
    assert op.n_dofs * 8 > 64 * 2**20
    x = torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda")
    r = torch.zeros_like(x)
    p = torch.zeros_like(x)
    res = torch.zeros(2, dtype=torch.float64, device="cuda")
    vp = lambda t: C.c_void_p(t.data_ptr())
    rc = L.lib().ufem_cg_iterate_static(op._h, L.F64, 1, vp(x), vp(r), vp(p), vp(res), None)
    assert rc == L.UFEM_EINVAL
    assert b"static workspace" in L.lib().ufem_last_error()
