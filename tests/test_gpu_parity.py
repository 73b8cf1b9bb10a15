"""GPU parity: the HIP operator against the FP64 oracle, element by element,
on the same seeded inputs.  FP64 within 1e-12 and FP32 within 1e-5 relative
to the largest entry; per term and for the whole operator; adjoint and
coefficient derivative; every small case again with the workgroups of each
launch capped (so that every workgroup takes many cell groups and line
batches in turn); the full-size workloads on sampled cells."""
import os
import sys

import numpy as np
import pytest

import ufem_inputs as ui
from oracle.operator import ALL, GP, NITSCHE, SIPG, VOL
from tests.helpers import SMALL_CASES, case_options, make_case, oracle_for

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
        opts = case_options(name)
        ora = oracle_for(wl, **opts)
        pl = Plan(Problem.from_workload(wl, **opts))
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


def _rows(v, cls, cells, nd):
    rank = np.cumsum(cls != 2) - 1
    return np.stack([v[rank[b] * nd:(rank[b] + 1) * nd] for b in cells])


def _row_err(got, ref):
    """max |got - ref| over the sampled rows relative to their largest entry"""
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def test_full_size_ball_sampled_rows(torch):
    """64^3 background cells, degree 3 (4.9M active DoF), the launch
    configuration of the benchmark; rows of sampled inside and cut cells,
    against the oracle evaluated here on those rows."""
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
    cls = pl.cells()
    assert _row_err(_rows(v, cls, cells, ora.nd), _rows(ref, ora.cls, cells, ora.nd)) < TOL64
    assert np.isfinite(np.linalg.norm(v))


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FULL = (["ball3d", "balls3d", "kappa3d"] + [f"sweep{p}" for p in range(1, 8)]
        + ["plane_p1_l0", "plane_p1_l9", "plane_p3_l0", "plane_p3_l1"])


def _full_workload(name):
    if name == "ball3d":
        return ui.ball3d(0)
    if name == "balls3d":
        return ui.balls3d(0)
    if name == "kappa3d":
        return ui.kappa3d(0)
    if name.startswith("plane_p"):
        p, layer = name[7:].split("_l")
        return ui.plane3d(int(layer), 0, n=128, degree=int(p))
    return ui.sweep3d(int(name[5:]), 0)


@pytest.mark.parametrize("name", FULL)
def test_full_size_sampled_rows_against_stored_oracle_rows(torch, name):
    """The full workloads (the ball at 64^3, p = 3; 20 balls at 128^3, p = 3;
    the kappa field at 48^3, p = 4; the degree sweep at about 2e7 active DoF,
    p = 1..7; the plane benchmark at 128^3, p = 1 and 3, cut-cell ratios 1,
    0.5 and 0.1) in the benchmark's launch configuration: FP64 and FP32
    applies, the adjoint pass and, for the ball and the kappa field,
    dL/dkappa, on the rows / points of sampled cells, against oracle values
    written by tests/golden/make_fullsize_rows.py for the same seeded
    inputs."""
    from paper_2404_07911_amd import Operator, Plan, Problem

    ref = np.load(os.path.join(GOLDEN, f"fullsize_{name}.npz"))
    wl, rng = _full_workload(name)
    _say(f"[{name} full size] plan")
    pl = Plan(Problem.from_workload(wl))
    n = pl.info["n_dofs"]
    assert n == int(ref["n_dofs"]) and wl.degree == int(ref["degree"])
    op = Operator(pl)
    u = ui.uniform_vector(rng, n)
    w = ui.uniform_vector(rng, n)
    cells = [int(b) for b in ref["cells"]]
    cls = pl.cells()
    nd = (wl.degree + 1) ** 3
    kap = None
    if name == "kappa3d":
        kap = torch.from_numpy(ui.kappa_field(pl.qp()[0])).cuda()
        op.set_kappa(kap)
    ud = torch.from_numpy(u).cuda()
    _say(f"[{name} full size] fp64 apply")
    v = op.apply(ud).cpu().numpy()
    e64 = _row_err(_rows(v, cls, cells, nd), ref["rows64"])
    _say(f"[{name} full size] fp32 apply")
    v32 = op.apply(ud.to(torch.float32)).cpu().numpy().astype(np.float64)
    e32 = _row_err(_rows(v32, cls, cells, nd), ref["rows32"])
    _say(f"[{name} full size] adjoint")
    atw, dk = op.apply_adjoint(torch.from_numpy(w).cuda(), ud)
    ea = _row_err(_rows(atw.cpu().numpy(), cls, cells, nd), ref["rows_adj"])
    _say(f"[{name} full size] errors fp64 {e64:.2e} fp32 {e32:.2e} adjoint {ea:.2e}")
    assert e64 < TOL64 and ea < TOL64 and e32 < TOL32, (e64, e32, ea)
    if "dk_idx" in ref:
        idx = ref["dk_idx"]
        ek = _row_err(dk.cpu().numpy()[idx], ref["dk_val"])
        _say(f"[{name} full size] dkappa {ek:.2e} on {idx.size} points")
        assert ek < TOL64, ek


@pytest.mark.parametrize("name", sorted(SMALL_CASES))
def test_multi_batch_paths(torch, name):
    """Every launch capped at 1 and at 3 workgroups: each workgroup then runs
    many cell groups of the structured kernels and many line batches of the
    cut-cell kernels (batch records and descriptors prefetched across
    batches, LDS reused), in both precisions, for the apply, the adjoint and
    dL/dkappa; the results equal the uncapped launches (one workgroup per
    batch or a persistent grid, by degree) bit for bit and the oracle within
    the tolerances."""
    wl, ora, pl, op, u, w = _setup(name)
    ud = torch.from_numpy(u).cuda()
    wd = torch.from_numpy(w).cuda()
    kap = torch.from_numpy(ui.kappa_field(ora.qp_physical_points())).cuda()

    def run():
        out = [op.apply(ud), op.apply(ud.to(torch.float32))]
        out += list(op.apply_adjoint(wd, ud))
        op.set_kappa(kap)
        out += [op.apply(ud)] + list(op.apply_adjoint(wd, ud))
        op.set_kappa(None)
        return out

    try:
        op.set_max_blocks(0)
        base = run()
        for cap in (1, 3):
            _say(f"[{name}] max_blocks {cap}")
            op.set_max_blocks(cap)
            got = run()
            for i, (a, b) in enumerate(zip(got, base)):
                assert torch.equal(a, b), (cap, i)
    finally:
        op.set_max_blocks(0)
        op.set_kappa(None)
    assert _rel(got[0].cpu().numpy(), ora.apply(u)) < TOL64
    assert _rel(got[5].cpu().numpy(), ora.apply(w, ALL, kap.cpu().numpy())) < TOL64


def test_adjoint_rejects_mismatched_outputs(torch):
    wl, ora, pl, op, u, w = _setup("disk2d_p2")
    ud = torch.from_numpy(u).cuda()
    wd = torch.from_numpy(w).cuda()
    with pytest.raises(TypeError):
        op.apply_adjoint(wd, ud, atw=torch.empty(ora.n_dofs, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        op.apply_adjoint(wd, ud, atw=torch.empty(ora.n_dofs - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        op.apply_adjoint(wd, ud, dkappa=torch.empty(op.n_qp, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        op.apply_adjoint(wd, ud, dkappa=torch.empty(op.n_qp + 3, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        op.apply_adjoint(wd, ud, atw=torch.empty(ora.n_dofs, dtype=torch.float64))


def test_dkappa_follows_the_term_mask(torch):
    """dL/dkappa of a masked operator covers the selected terms only (the
    derivative of w^T A_mask(kappa) u)."""
    from oracle.operator import NITSCHE as ON, SIPG as OS, VOL as OV

    from paper_2404_07911_amd import TERM_ALL

    wl, ora, pl, op, u, w = _setup("ball3d_p2")
    ud = torch.from_numpy(u).cuda()
    wd = torch.from_numpy(w).cuda()
    full = ora.dkappa(w, u)
    seg = ora.layout()["segments"]
    parts = {OV: [(seg[0], seg[2])], OS: [(seg[2], seg[4])], ON: [(seg[4], seg[5])]}
    try:
        for mask in (OV, OS, ON, OV | ON):
            op.set_terms(mask)
            dk = op.apply_adjoint(wd, ud)[1].cpu().numpy()
            ref = np.zeros_like(full)
            for bit, rngs in parts.items():
                if mask & bit:
                    for a, b in rngs:
                        ref[a:b] = full[a:b]
            assert np.abs(dk - ref).max() <= 1e-12 * np.abs(full).max(), mask
    finally:
        op.set_terms(TERM_ALL)


@pytest.mark.parametrize("name", ["ball3d_p3", "disk2d_p2", "balls3d_p2", "plane3d_p2", "union3d_fallback"])
def test_apply_with_imported_oracle_quadrature(torch, name):
    """setup(..., quadrature): the oracle's own cut rules (q = p + 2 points
    per 1D piece, not the plan's q = p + 1) imported into the plan; the
    operator then equals the oracle built on the same rules, apply, FP32
    apply and the adjoint pass with a kappa field."""
    from paper_2404_07911_amd import Operator, Plan, Problem
    from tests.helpers import oracle_cut_rules

    wl, rng = make_case(name)
    opts = case_options(name)
    ora = oracle_for(wl, q=wl.degree + 2, **opts)
    pl = Plan(Problem.from_workload(wl, **opts))
    pl.import_quadrature(*oracle_cut_rules(ora))
    op = Operator(pl)
    u = ui.uniform_vector(rng, ora.n_dofs)
    w = ui.uniform_vector(rng, ora.n_dofs)
    ud = torch.from_numpy(u).cuda()
    _say(f"[{name}] imported rules")
    assert _rel(op.apply(ud).cpu().numpy(), ora.apply(u)) < TOL64
    u32 = u.astype(np.float32)
    v32 = op.apply(torch.from_numpy(u32).cuda()).cpu().numpy().astype(np.float64)
    assert _rel(v32, ora.apply(u32.astype(np.float64))) < TOL32
    kap = ui.kappa_field(ora.qp_physical_points())
    op.set_kappa(torch.from_numpy(kap).cuda())
    atw, dk = op.apply_adjoint(torch.from_numpy(w).cuda(), ud)
    assert _rel(atw.cpu().numpy(), ora.apply(w, ALL, kap)) < TOL64
    assert _rel(dk.cpu().numpy(), ora.dkappa(w, u)) < TOL64


@pytest.mark.parametrize("name", ["ball3d_p1", "ball3d_p3", "disk2d_p2", "balls3d_p2", "plane3d_p2",
                                  "union3d_fallback", "ball3d_p2_vgp", "disk2d_p7"])
def test_mixed_evaluation(torch, name):
    """The mixed evaluation (the cut cells' volume and interface terms as
    precomputed element matrices, the rest matrix-free) against the oracle:
    FP64 and FP32 applies per term and whole, and the adjoint pass with a
    kappa field (the matrices follow set_terms and set_kappa); back to the
    matrix-free evaluation afterwards."""
    from paper_2404_07911_amd import TERM_ALL

    wl, ora, pl, op, u, w = _setup(name)
    ud = torch.from_numpy(u).cuda()
    free = op.apply(ud).clone()
    try:
        _say(f"[{name}] mixed")
        op.set_mixed(True)
        for mask in (VOL, NITSCHE, ALL):
            op.set_terms(mask)
            assert _rel(op.apply(ud).cpu().numpy(), ora.apply(u, mask)) < TOL64, mask
        op.set_terms(TERM_ALL)
        u32 = u.astype(np.float32)
        v32 = op.apply(torch.from_numpy(u32).cuda()).cpu().numpy().astype(np.float64)
        assert _rel(v32, ora.apply(u32.astype(np.float64))) < TOL32
        kap = ui.kappa_field(ora.qp_physical_points())
        op.set_kappa(torch.from_numpy(kap).cuda())
        atw, dk = op.apply_adjoint(torch.from_numpy(w).cuda(), ud)
        assert _rel(atw.cpu().numpy(), ora.apply(w, ALL, kap)) < TOL64
        assert _rel(dk.cpu().numpy(), ora.dkappa(w, u)) < TOL64
    finally:
        op.set_mixed(False)
        op.set_terms(TERM_ALL)
        op.set_kappa(None)
    assert torch.equal(op.apply(ud), free)


CG_CASES = ["disk2d_p2", "disk2d_p4", "ball3d_p1", "ball3d_p2", "ball3d_p3", "balls3d_p2", "plane3d_p2",
            "ball3d_p2_vgp", "union3d_fallback"]
_CG_CACHE = {}


def _setup_cg(name):
    if name not in _CG_CACHE:
        from oracle.operator import UnfittedCG
        from paper_2404_07911_amd import Operator, Plan, Problem

        wl, rng = make_case(name)
        opts = case_options(name)
        ora = UnfittedCG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, wl.lo, wl.hi, plane=wl.plane, **opts)
        op = Operator(Plan(Problem.from_workload(wl, space="cg", **opts)))
        u = ui.uniform_vector(rng, ora.n_dofs)
        w = ui.uniform_vector(rng, ora.n_dofs)
        _CG_CACHE[name] = (wl, ora, op, u, w)
    return _CG_CACHE[name]


@pytest.mark.parametrize("name", CG_CASES)
def test_continuous_space(torch, name):
    """The continuous space (FE_Q): P^T A_cell P on the GPU (node gather,
    cell-DoF operator without SIPG, deterministic node sums) against the
    oracle, per term and whole in FP64, FP32, the adjoint pass and dL/dkappa
    with a kappa field, launches capped at 2 workgroups, and the mixed
    evaluation; repeated applies bit-identical."""
    from paper_2404_07911_amd import TERM_ALL

    wl, ora, op, u, w = _setup_cg(name)
    ud = torch.from_numpy(u).cuda()
    _say(f"[{name}] continuous space")
    for mask in (VOL, NITSCHE, GP, ALL):
        op.set_terms(mask)
        assert _rel(op.apply(ud).cpu().numpy(), ora.apply(u, mask)) < TOL64, mask
    op.set_terms(TERM_ALL)
    v = op.apply(ud)
    assert torch.equal(v, op.apply(ud))
    u32 = u.astype(np.float32)
    v32 = op.apply(torch.from_numpy(u32).cuda()).cpu().numpy().astype(np.float64)
    assert _rel(v32, ora.apply(u32.astype(np.float64))) < TOL32
    kap = ui.kappa_field(ora.dg.qp_physical_points())
    op.set_kappa(torch.from_numpy(kap).cuda())
    try:
        atw, dk = op.apply_adjoint(torch.from_numpy(w).cuda(), ud)
        assert _rel(atw.cpu().numpy(), ora.apply(w, ALL, kap)) < TOL64
        assert _rel(dk.cpu().numpy(), ora.dkappa(w, u)) < TOL64
        op.set_max_blocks(2)
        assert _rel(op.apply(ud).cpu().numpy(), ora.apply(u, ALL, kap)) < TOL64
        op.set_max_blocks(0)
        op.set_mixed(True)
        assert _rel(op.apply(ud).cpu().numpy(), ora.apply(u, ALL, kap)) < TOL64
    finally:
        op.set_mixed(False)
        op.set_max_blocks(0)
        op.set_kappa(None)


def test_continuous_space_solve(torch):
    """Device CG on the continuous space to 1e-10 (residual re-checked with
    the oracle), FP64 and FP32-inner defect correction."""
    from paper_2404_07911_amd.solvers import device_cg, device_defect_correction

    wl, ora, op, u, w = _setup_cg("ball3d_p2")
    b = op.apply(torch.from_numpy(u).cuda())
    bh = b.cpu().numpy()
    x, info = device_cg(op, b, torch.zeros_like(b), rtol=1e-10, maxiter=20000, chunk=16)
    assert info["converged"], info
    assert np.linalg.norm(bh - ora.apply(x.cpu().numpy())) < 2e-10 * np.linalg.norm(bh)
    x2, info2 = device_defect_correction(op, b, tol=1e-10, inner_rtol=1e-4)
    assert info2["converged"], info2
    assert np.linalg.norm(bh - ora.apply(x2.cpu().numpy())) < 2e-10 * np.linalg.norm(bh)
