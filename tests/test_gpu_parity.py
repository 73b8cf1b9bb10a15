"""GPU parity: the HIP operator against the FP64 oracle, element by element,
on the same seeded inputs.  FP64 within 1e-12 and FP32 within 1e-5 relative
to the largest entry; per term and for the whole operator; adjoint and
coefficient derivative; the full 64^3 degree-3 ball on sampled cells."""
import sys

import numpy as np
import pytest

import ufem_inputs as ui
from oracle.operator import ALL, GP, NITSCHE, SIPG, VOL
from tests.helpers import SMALL_CASES, make_case, oracle_for

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


_CACHE = {}


def _setup(name):
    if name not in _CACHE:
        from paper_2404_07911_amd import Operator, Plan, Problem

        wl, rng = make_case(name)
        ora = oracle_for(wl)
        pl = Plan(Problem.from_workload(wl))
        op = Operator(pl)
        u = ui.uniform_vector(rng, ora.n_dofs)
        w = ui.uniform_vector(rng, ora.n_dofs)
        _CACHE[name] = (wl, ora, pl, op, u, w)
    return _CACHE[name]


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", sorted(SMALL_CASES))
def test_apply_fp64_per_term_and_full(torch, name):
    from paper_2404_07911_amd import TERM_ALL

    wl, ora, pl, op, u, w = _setup(name)
    ud = torch.from_numpy(u).cuda()
    for mask in (VOL, SIPG, NITSCHE, GP, ALL):
        _say(f"[{name}] fp64 mask {mask}")
        op.set_terms(mask)
        v = op.apply(ud).cpu().numpy()
        ref = ora.apply(u, mask)
        err = _rel(v, ref)
        assert err < TOL64, (name, mask, err)
    op.set_terms(TERM_ALL)


@pytest.mark.parametrize("name", sorted(SMALL_CASES))
def test_apply_fp32(torch, name):
    wl, ora, pl, op, u, w = _setup(name)
    _say(f"[{name}] fp32")
    u32 = u.astype(np.float32)
    v = op.apply(torch.from_numpy(u32).cuda()).cpu().numpy().astype(np.float64)
    ref = ora.apply(u32.astype(np.float64))
    assert _rel(v, ref) < TOL32


@pytest.mark.parametrize("name", ["disk2d_p2", "disk2d_p7", "ball3d_p2", "ball3d_p3", "ball3d_p5", "ball3d_p7",
                                  "balls3d_p2"])
def test_adjoint_and_dkappa_with_variable_kappa(torch, name):
    wl, ora, pl, op, u, w = _setup(name)
    _say(f"[{name}] adjoint")
    kap = ui.kappa_field(ora.qp_physical_points())
    op.set_kappa(torch.from_numpy(kap).cuda())
    try:
        v = op.apply(torch.from_numpy(u).cuda()).cpu().numpy()
        assert _rel(v, ora.apply(u, ALL, kap)) < TOL64
        atw, dk = op.apply_adjoint(torch.from_numpy(w).cuda(), torch.from_numpy(u).cuda())
        atw = atw.cpu().numpy()
        dk = dk.cpu().numpy()
        assert _rel(atw, ora.apply(w, ALL, kap)) < TOL64
        assert _rel(dk, ora.dkappa(w, u)) < TOL64
        # dot test <w, A u> = <A^T w, u>
        assert abs(w @ v - atw @ u) < 1e-12 * abs(w @ v) + 1e-12
    finally:
        op.set_kappa(None)


@pytest.mark.parametrize("name", sorted(SMALL_CASES))
def test_adjoint_and_dkappa_constant_kappa(torch, name):
    """kappa = 1: A^T w and the per-point coefficient derivative."""
    wl, ora, pl, op, u, w = _setup(name)
    _say(f"[{name}] adjoint kappa=1")
    atw, dk = op.apply_adjoint(torch.from_numpy(w).cuda(), torch.from_numpy(u).cuda())
    assert _rel(atw.cpu().numpy(), ora.apply(w)) < TOL64
    assert _rel(dk.cpu().numpy(), ora.dkappa(w, u)) < TOL64
    atw32, dk32 = op.apply_adjoint(torch.from_numpy(w.astype(np.float32)).cuda(),
                                   torch.from_numpy(u.astype(np.float32)).cuda())
    w64, u64 = w.astype(np.float32).astype(np.float64), u.astype(np.float32).astype(np.float64)
    assert _rel(atw32.cpu().numpy().astype(np.float64), ora.apply(w64)) < TOL32
    assert _rel(dk32.cpu().numpy().astype(np.float64), ora.dkappa(w64, u64)) < TOL32


@pytest.mark.parametrize("name", ["ball3d_p3", "disk2d_p2", "balls3d_p2"])
def test_apply_stages_compose(torch, name):
    """The kernel stages, one call each, give ufem_apply bit for bit, on the
    kappa = 1 path (Kronecker kernel, then volume/interface and cut-face
    lines) and with a kappa field (structured terms per Gauss point)."""
    from paper_2404_07911_amd import PART_CUT, PART_INSIDE, UfemError

    wl, ora, pl, op, u, w = _setup(name)
    ud = torch.from_numpy(u).cuda()
    kap = torch.from_numpy(ui.kappa_field(ora.qp_physical_points())).cuda()
    try:
        for k in (None, kap):
            _say(f"[{name}] stages, kappa {'field' if k is not None else '1'}")
            op.set_kappa(k)
            full = op.apply(ud)
            for parts in ((1, 2, 4, 8), (3, 4, 8), (1, 2, 12)):
                v = torch.full_like(ud, float("nan"))
                for part in parts:
                    op.apply_part(part, ud, v)
                assert torch.equal(v, full), parts
            v = torch.full_like(ud, float("nan"))
            op.apply_part(PART_INSIDE, ud, v)
            op.apply_part(PART_CUT, ud, v)
            assert torch.equal(v, full)
        for bad in (0, 16, -1):
            with pytest.raises(UfemError):
                op.apply_part(bad, ud, v)
    finally:
        op.set_kappa(None)


def test_apply_is_repeatable_and_overwrites(torch):
    wl, ora, pl, op, u, w = _setup("ball3d_p3")
    ud = torch.from_numpy(u).cuda()
    v = torch.full_like(ud, float("nan"))
    op.apply(ud, v)
    a = v.clone()
    op.apply(ud, v)
    assert torch.equal(a, v)
    assert torch.isfinite(v).all()


def test_apply_rejects_aliasing(torch):
    from paper_2404_07911_amd import UfemError

    wl, ora, pl, op, u, w = _setup("disk2d_p2")
    ud = torch.from_numpy(u).cuda()
    with pytest.raises(UfemError):
        op.apply(ud, ud)


def test_full_size_ball_sampled_rows(torch):
    """64^3 background cells, degree 3 (4.9M active DoF), the launch
    configuration of the benchmark; rows of sampled inside and cut cells."""
    from paper_2404_07911_amd import Operator, Plan, Problem

    wl, rng = ui.ball3d(0)
    _say("[ball3d 64^3] plan")
    pl = Plan(Problem.from_workload(wl))
    op = Operator(pl)
    u = ui.uniform_vector(rng, pl.info["n_dofs"])
    _say("[ball3d 64^3] apply")
    v = op.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    ora = oracle_for(wl)
    pick = np.random.default_rng(7)
    cells = list(pick.choice(ora.inside_cells, 6, replace=False)) + list(pick.choice(ora.cut_cells, 10, replace=False))
    _say("[ball3d 64^3] oracle rows")
    ref = ora.apply(u, ALL, None, cells=cells)
    for b in cells:
        r = ora.rank[b]
        sl = slice(r * ora.nd, (r + 1) * ora.nd)
        assert _rel(v[sl], ref[sl]) < 1e-11, b
    s = np.linalg.norm(v)
    assert np.isfinite(s)
