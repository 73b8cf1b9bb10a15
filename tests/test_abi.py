"""CPU tests of the C ABI: the library loads and exports every declared entry
point, the host plan equals the oracle's classification, faces and
quadrature, and invalid arguments are rejected."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import ufem_inputs as ui
from tests.helpers import SMALL_CASES, case_options, make_case, oracle_for, oracle_qp_arrays

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2404_07911_amd import _lib

    return _lib


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "ufem.h")).read()
    declared = sorted(set(re.findall(r"\b(ufem_[a-z_0-9]+)\s*\(", hdr)))
    assert len(declared) >= 15
    L = _lib().lib()
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(_lib().exported_symbols()) == declared


@pytest.mark.parametrize("name", sorted(SMALL_CASES))
def test_plan_matches_oracle(name):
    from paper_2404_07911_amd import Plan, Problem

    wl, _ = make_case(name)
    opts = case_options(name)
    pl = Plan(Problem.from_workload(wl, **opts))
    op = oracle_for(wl, **opts)
    assert np.array_equal(pl.cells(), op.cls)
    kinds = {"str": 0, "cut": 1, "none": 2}
    of = np.array([(a, b, c, kinds[k], int(g)) for a, b, c, k, g in op.faces], dtype=np.int32).reshape(-1, 5)
    assert np.array_equal(pl.faces(), of)
    L = op.layout()
    assert list(pl.info["seg"]) == list(L["segments"])
    assert pl.info["n_dofs"] == op.n_dofs
    xyz, ref, w, nrm = pl.qp()
    oref, ow, onrm = oracle_qp_arrays(op)
    assert np.abs(ref - oref).max() < 1e-13
    assert np.abs(w - ow).max() < 1e-13 * max(1.0, np.abs(ow).max())
    assert np.abs(nrm - onrm).max() < 1e-13
    assert np.abs(xyz - op.qp_physical_points()).max() < 1e-13
    assert pl.info["n_fallback"] == op.saye.n_fallback


def test_edge_cases_reach_their_paths():
    """The fallback cases hit the subdivision limit; in the tangent cases the
    sphere touches mesh planes at mesh vertices only."""
    from paper_2404_07911_amd import Plan, Problem

    for name in ("union2d_fallback", "union3d_fallback"):
        wl, _ = make_case(name)
        pl = Plan(Problem.from_workload(wl, **case_options(name)))
        assert pl.info["n_fallback"] > 0, name
    for name in ("tangent2d", "tangent3d"):
        wl, _ = make_case(name)
        pl = Plan(Problem.from_workload(wl))
        assert pl.info["n_fallback"] == 0
        cls = pl.cells()
        n = wl.n
        # the sphere touches the plane x = 0.5 at (0.5, 0, 0), a mesh vertex:
        # the cell beyond it is outside (distance exactly R), the one before
        # is cut, and the pieces of zero measure are dropped (no zero weight)
        beyond = 6 + n * (n // 2) + (n * n * (n // 2) if wl.dim == 3 else 0)
        assert cls[beyond] == 2 and cls[beyond - 1] == 1
        _, _, w, _ = pl.qp()
        assert (w > 0).all()


def test_plan_full_size_ball_counts():
    """The 64^3 degree-3 ball plan builds on the host in seconds and its
    counts match the oracle's classification."""
    from paper_2404_07911_amd import Plan, Problem
    from oracle.geometry import Balls, Mesh, classify_cells

    wl, _ = ui.ball3d(0)
    pl = Plan(Problem.from_workload(wl))
    cls = classify_cells(Mesh(3, 64), Balls(wl.centers, wl.radii))
    assert np.array_equal(pl.cells(), cls)
    assert pl.info["n_active"] == int(np.sum(cls != 2))
    assert pl.info["n_dofs"] == pl.info["n_active"] * 64
    assert pl.info["n_fallback"] == 0


def _problem(**over):
    from paper_2404_07911_amd import Problem

    base = dict(dim=3, n=8, degree=2, centers=np.zeros((1, 3)), radii=np.array([0.5]))
    base.update(over)
    return Problem(**base)


@pytest.mark.parametrize(
    "over",
    [
        dict(degree=0),
        dict(degree=8),
        dict(dim=4, centers=np.zeros((1, 4))),
        dict(n=1),
        dict(radii=np.array([-0.5])),
        dict(q_cut=99),
        dict(lo=1.0, hi=-1.0),
        dict(centers=np.full((1, 3), 5.0)),  # no active cell
    ],
)
def test_plan_rejects_bad_problems(over):
    from paper_2404_07911_amd import Plan, UfemError

    with pytest.raises(UfemError) as e:
        Plan(_problem(**over))
    assert e.value.code in (-1, -4)


def test_null_arguments_are_rejected():
    L = _lib()
    lib = L.lib()
    assert lib.ufem_plan_create(None, None) == L.UFEM_EINVAL
    assert lib.ufem_plan_info(None, None) == L.UFEM_EINVAL
    assert lib.ufem_apply(None, 0, None, None, None) == L.UFEM_EINVAL
    assert lib.ufem_apply_adjoint(None, 0, None, None, None, None, None) == L.UFEM_EINVAL
    assert lib.ufem_set_terms(None, 15) == L.UFEM_EINVAL
    assert lib.ufem_set_kappa(None, 0, None, None) == L.UFEM_EINVAL
    assert lib.ufem_dot(0, 10, None, None, None, None) == L.UFEM_EINVAL
    assert lib.ufem_axpby(0, 10, 1.0, None, 1.0, None, None) == L.UFEM_EINVAL
    assert lib.ufem_cast(0, 1, 10, None, None, None) == L.UFEM_EINVAL
    assert lib.ufem_cast(0, 2, 10, C.c_void_p(16), C.c_void_p(4096), None) == L.UFEM_EINVAL
    assert lib.ufem_cg_iterate(None, 0, 1, None, None, None, None, None, None) == L.UFEM_EINVAL
    assert lib.ufem_apply_part(None, 0, 15, None, None, None) == L.UFEM_EINVAL
    assert b"ufem_" in lib.ufem_last_error()


def test_setup_without_gpu_fails_cleanly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2404_07911_amd import Plan, UfemError

    pl = Plan(_problem())
    L = _lib()
    h = C.c_void_p()
    rc = L.lib().ufem_setup(pl.handle, 0, None, 0, C.byref(h))
    assert rc in (L.UFEM_EHIP, L.UFEM_EINVAL)
    assert not h.value


@pytest.mark.parametrize("name", ["ball3d_p3", "disk2d_p2", "balls3d_p2", "plane3d_p2", "union3d_fallback"])
def test_import_quadrature_replaces_the_cut_rules(name):
    """The oracle's rules with q = p + 2 points per 1D piece (not the plan's
    own q = p + 1) go into the plan: its counts, kappa layout and exported
    points are then exactly the oracle's."""
    from paper_2404_07911_amd import Plan, Problem
    from tests.helpers import oracle_cut_rules

    wl, _ = make_case(name)
    opts = case_options(name)
    pl = Plan(Problem.from_workload(wl, **opts))
    ora = oracle_for(wl, q=wl.degree + 2, **opts)
    pl.import_quadrature(*oracle_cut_rules(ora))
    L = ora.layout()
    assert list(pl.info["seg"]) == list(L["segments"])
    xyz, ref, w, nrm = pl.qp()
    oref, ow, onrm = oracle_qp_arrays(ora)
    seg = L["segments"]
    cut = np.r_[seg[1]:seg[2], seg[3]:seg[5]]  # imported: bit for bit
    face_axis = np.abs(ref[cut] - oref[cut]).max(axis=1) if cut.size else np.zeros(0)
    assert np.array_equal(w[cut], ow[cut]) and np.array_equal(nrm[cut], onrm[cut])
    assert (face_axis == 0).all()
    # the tensor rules of the plan's own (structured) segments agree to rounding
    assert np.abs(w - ow).max() < 1e-15 and np.abs(ref - oref).max() < 1e-15
    assert pl.info["max_qp_cut_cell"] == max(L["vol"][b][1] for b in ora.cut_cells)


def test_import_quadrature_rejects_bad_rules():
    from paper_2404_07911_amd import Plan, Problem, UfemError
    from tests.helpers import oracle_cut_rules

    wl, _ = make_case("disk2d_p2")
    pl = Plan(Problem.from_workload(wl))
    before = dict(pl.info)
    vc, fc, sc, ref, w, nrm = oracle_cut_rules(oracle_for(wl))
    bad = [
        (np.where(np.arange(vc.size) == 0, -1, vc), fc, sc, ref, w, nrm),
        (vc, fc, sc, np.where(np.arange(ref.size).reshape(ref.shape) == 0, 1.5, ref), w, nrm),
        (vc, fc, sc, ref, np.where(np.arange(w.size) == 3, -0.1, w), nrm),
        (vc, fc, sc, ref, np.where(np.arange(w.size) == 3, np.nan, w), nrm),
    ]
    for args in bad:
        with pytest.raises((UfemError, ValueError)):
            pl.import_quadrature(*args)
    # a null pointer through the ABI
    L = _lib()
    assert L.lib().ufem_plan_import_quadrature(pl.handle, None, None, None, None, None, None) == L.UFEM_EINVAL
    inf = L.ufem_info()
    L.check(L.lib().ufem_plan_info(pl.handle, C.byref(inf)))
    assert inf.as_dict() == before


@pytest.mark.parametrize("name", ["disk2d_p2", "ball3d_p2", "balls3d_p2", "plane3d_p2", "ball3d_p2_vgp"])
def test_continuous_space_node_count(name):
    """The continuous space's DoFs: the Gauss-Lobatto nodes of the active
    cells on the node lattice (the oracle's count); the cell-DoF layout and
    the quadrature stay those of the discontinuous plan."""
    from oracle.operator import UnfittedCG
    from paper_2404_07911_amd import Plan, Problem

    wl, _ = make_case(name)
    opts = case_options(name)
    pl = Plan(Problem.from_workload(wl, space="cg", **opts))
    dg = Plan(Problem.from_workload(wl, **opts))
    o = UnfittedCG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, wl.lo, wl.hi, plane=wl.plane, **opts)
    assert pl.info["n_dofs"] == o.n_dofs
    assert pl.info["n_cell_dofs"] == dg.info["n_dofs"] == o.dg.n_dofs
    assert pl.info["seg"] == dg.info["seg"]
