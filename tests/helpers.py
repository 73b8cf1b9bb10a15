"""Shared test helpers: build the oracle and the product plan from the same
seeded workload, and flatten the oracle's quadrature into kappa order."""
import numpy as np

import ufem_inputs as ui
from oracle.geometry import INSIDE
from oracle.operator import UnfittedDG


def oracle_for(wl, **kw):
    return UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, wl.lo, wl.hi, **kw)


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
}


def make_case(name):
    fn, kw = SMALL_CASES[name]
    return fn(**kw)
