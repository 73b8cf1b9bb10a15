"""Shared test helpers: build the oracle and the product plan from the same
seeded workload, and flatten the oracle's quadrature into kappa order."""
import numpy as np

import ufem_inputs as ui
from oracle.geometry import INSIDE
from oracle.operator import UnfittedDG


def oracle_for(wl, **kw):
    return UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, wl.lo, wl.hi, plane=wl.plane, **kw)


def oracle_qp_arrays(op):
    """Reference coordinates (faces: in the lower cell, on its upper face),
    reference weights and normals of every quadrature point, kappa order."""
    L = op.layout()
    n = L["n_qp"]
    d = op.dim
    ref = np.zeros((n, d))
    w = np.zeros(n)
    nrm = np.zeros((n, d))
    for b, (o, m) in L["vol"].items():
        if op.cls[b] == INSIDE:
            xi, wq = op.full_cell_rule()
        else:
            xi, wq = op.cell_rule(b)[:2]
        ref[o : o + m] = xi
        w[o : o + m] = wq
    for fi, (o, m) in L["face"].items():
        bm, bp, a, kind, gp = op.faces[fi]
        xf, wf = op.face_rule(fi)
        ref[o : o + m] = op._face_points(xf, a, 1.0)
        w[o : o + m] = wf
    for b, (o, m) in L["surf"].items():
        _, _, xs, ws, ns = op.cell_rule(b)
        ref[o : o + m] = xs
        w[o : o + m] = ws
        nrm[o : o + m] = ns
    return ref, w, nrm


SMALL_CASES = {
    # name: (factory, kwargs)
    "disk2d_p2": (ui.disk2d, dict(seed=0)),
    "disk2d_p1": (ui.disk2d, dict(seed=1, n=12, degree=1)),
    "disk2d_p4": (ui.disk2d, dict(seed=2, n=10, degree=4)),
    "ball3d_p1": (ui.ball3d, dict(seed=0, n=10, degree=1)),
    "ball3d_p2": (ui.ball3d, dict(seed=1, n=10, degree=2)),
    "ball3d_p3": (ui.ball3d, dict(seed=2, n=12, degree=3)),
    "ball3d_p4": (ui.ball3d, dict(seed=3, n=8, degree=4)),
    "balls3d_p2": (ui.balls3d, dict(seed=0, n=16, degree=2, n_balls=5)),
    "balls3d_p3": (ui.balls3d, dict(seed=4, n=12, degree=3, n_balls=3)),
    "ball3d_p5": (ui.ball3d, dict(seed=5, n=5, degree=5)),
    "ball3d_p6": (ui.ball3d, dict(seed=6, n=5, degree=6)),
    "ball3d_p7": (ui.ball3d, dict(seed=7, n=5, degree=7)),
    "disk2d_p7": (ui.disk2d, dict(seed=7, n=8, degree=7)),
    # two balls whose intersection curve has both centres on opposite sides
    # along every axis: no height direction exists near it, and with no
    # subdivision allowed the cells there take the tensor rule filtered by
    # phi < 0 (the fallback of the dimension-reduction rule)
    "union2d_fallback": (ui.custom, dict(dim=2, n=12, degree=3, centers=[[-0.31, -0.29], [0.3, 0.32]],
                                         radii=[0.5, 0.5], seed=21)),
    "union3d_fallback": (ui.custom, dict(dim=3, n=8, degree=2,
                                         centers=[[-0.31, -0.29, -0.3], [0.3, 0.32, 0.29]],
                                         radii=[0.55, 0.55], seed=22)),
    # degenerate cuts: a sphere centred on a mesh vertex whose radius is a
    # multiple of h touches six mesh planes at single points and passes
    # through mesh vertices (tangent faces carry no SIPG term, and the cells
    # beyond them are outside)
    "tangent3d": (ui.custom, dict(dim=3, n=8, degree=2, centers=[[0.0, 0.0, 0.0]], radii=[0.5], seed=23)),
    "tangent2d": (ui.custom, dict(dim=2, n=8, degree=3, centers=[[0.0, 0.0]], radii=[0.5], seed=24)),
    # plane level sets (the plane benchmark's geometry): a tilted plane
    # through the box, and the benchmark's near-horizontal plane in one layer
    "plane3d_p2": (ui.plane, dict(dim=3, n=8, degree=2, normal=[0.3, -0.5, 0.81], offset=0.07, seed=25)),
    "plane2d_p3": (ui.plane, dict(dim=2, n=10, degree=3, normal=[0.6, -0.8], offset=0.05, seed=26)),
    "plane3d_layer_p1": (ui.plane3d, dict(layer=3, n=12, degree=1, seed=27)),
    # the volume ghost penalty (Section 2.2): stable-neighbour patches, and
    # every face of a cut cell (all-neighbours strategy)
    "ball3d_p2_vgp": (ui.ball3d, dict(seed=8, n=10, degree=2)),
    "ball3d_p3_vgp": (ui.ball3d, dict(seed=9, n=8, degree=3)),
    "disk2d_p3_vgp": (ui.disk2d, dict(seed=10, n=12, degree=3)),
    "balls3d_p2_vgp_all": (ui.balls3d, dict(seed=11, n=12, degree=2, n_balls=4)),
}

# options of the plan and of the oracle beyond the workload (same keywords)
CASE_OPTIONS = {
    "union2d_fallback": dict(max_depth=0),
    "union3d_fallback": dict(max_depth=0),
    "ball3d_p2_vgp": dict(gp_kind="volume"),
    "ball3d_p3_vgp": dict(gp_kind="volume"),
    "disk2d_p3_vgp": dict(gp_kind="volume"),
    "balls3d_p2_vgp_all": dict(gp_kind="volume_all"),
}


def make_case(name):
    fn, kw = SMALL_CASES[name]
    return fn(**kw)


def case_options(name):
    return dict(CASE_OPTIONS.get(name, {}))


def oracle_cut_rules(op):
    """The oracle's cut rules in the layout of ufem_plan_import_quadrature:
    counts per cut cell (volume), cut face and cut cell (interface), then the
    reference points, weights and normals of those three kappa segments."""
    L = op.layout()
    ref, w, nrm = oracle_qp_arrays(op)
    seg = L["segments"]
    vc = [L["vol"][b][1] for b in op.cut_cells]
    fc = [L["face"][fi][1] for fi, f in enumerate(op.faces) if f[3] == "cut"]
    sc = [L["surf"][b][1] for b in op.cut_cells]
    sl = np.r_[seg[1]:seg[2], seg[3]:seg[5]]
    return np.array(vc), np.array(fc), np.array(sc), ref[sl], w[sl], nrm[sl]
