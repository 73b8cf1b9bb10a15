"""Pins of the oracle's plane level set (the plane benchmark of Section 5.2):
the dimension-reduction rules of cells, faces and the interface cut by a
plane against exact polynomial moments of the clipped polytopes.

The reference moments are computed independently of the oracle: the box is
clipped by the half space n . x < c (vertices of the polytope), the polytope
is split into simplices (fan from its centroid over the facets of its convex
hull), and each simplex is integrated by a collapsed (Duffy) Gauss product
rule, which is exact for polynomials once it has enough points.  The rules of
the oracle are exact too, because the height function of a plane is linear:
with q Gauss points per 1D piece, monomials of degree up to 2q - d on a cut
cell, 2q - d + 1 on the interface and 2q - d + 1 on a cut face (d - 1
dimensions) are integrated without error (each dimension of the reduction
adds one to the degree of the integrand through the linear piece limits).
"""
import itertools
import math

import numpy as np
import pytest
from scipy.spatial import ConvexHull

from oracle.basis import gauss_legendre
from oracle.geometry import CUT, INSIDE, OUTSIDE, Mesh, Plane, box_class, classify_cells
from oracle.quadrature import SayeQuadrature


def _simplex_moment(V, alpha, npt=5):
    """integral over the simplex with vertices V (m+1 rows, m columns) of
    prod x_a^alpha_a, by the collapsed Gauss rule on [0, 1]^m"""
    m = V.shape[1]
    gx, gw = gauss_legendre(npt)
    total = 0.0
    for idx in itertools.product(range(npt), repeat=m):
        u = [gx[i] for i in idx]
        w = float(np.prod([gw[i] for i in idx]))
        # barycentric coordinates of the collapsed map and its Jacobian
        lam = np.zeros(m + 1)
        rest = 1.0
        jac = 1.0
        for j in range(m):
            lam[j] = rest * u[j]
            jac *= (1.0 - u[j]) ** (m - 1 - j)
            rest *= 1.0 - u[j]
        lam[m] = rest
        x = lam @ V
        total += w * jac * float(np.prod([x[a] ** alpha[a] for a in range(m)]))
    J = V[1:] - V[0]
    return total * abs(np.linalg.det(J))


def _clip_box(lo, hi, n, c):
    """vertices of {x in [lo, hi] : n . x <= c}"""
    d = len(lo)
    corners = [np.array([hi[a] if (b >> a) & 1 else lo[a] for a in range(d)]) for b in range(2**d)]
    pts = [x for x in corners if np.dot(n, x) <= c]
    for i, x in enumerate(corners):
        for j in range(i + 1, len(corners)):
            y = corners[j]
            if np.count_nonzero(x != y) != 1:
                continue
            fx, fy = np.dot(n, x) - c, np.dot(n, y) - c
            if fx * fy < 0:
                pts.append(x + fx / (fx - fy) * (y - x))
    return np.array(pts)


def _polytope_moment(P, alpha):
    d = P.shape[1]
    if d == 1:
        a, b = P.min(), P.max()
        return (b ** (alpha[0] + 1) - a ** (alpha[0] + 1)) / (alpha[0] + 1)
    hull = ConvexHull(P)
    cen = P.mean(axis=0)
    return sum(_simplex_moment(np.vstack([cen, P[s]]), alpha) for s in hull.simplices)


def _section_moment(lo, hi, n, c, alpha):
    """integral over {x in [lo, hi] : n . x = c} (surface measure)"""
    d = len(lo)
    corners = [np.array([hi[a] if (b >> a) & 1 else lo[a] for a in range(d)]) for b in range(2**d)]
    pts = []
    for i, x in enumerate(corners):
        for j in range(i + 1, len(corners)):
            y = corners[j]
            if np.count_nonzero(x != y) != 1:
                continue
            fx, fy = np.dot(n, x) - c, np.dot(n, y) - c
            if fx * fy < 0:
                pts.append(x + fx / (fx - fy) * (y - x))
    P = np.array(pts)
    if len(P) < d:  # the plane touches the box at a corner or edge only
        return 0.0
    if d == 2:
        a, b = P[0], P[1]
        gx, gw = gauss_legendre(8)
        L = float(np.linalg.norm(b - a))
        return sum(w * L * float(np.prod((a + t * (b - a)) ** np.array(alpha))) for t, w in zip(gx, gw))
    # 3D: the convex polygon, ordered by angle in the plane, fan from its centroid
    cen = P.mean(axis=0)
    e1 = P[0] - cen
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    ang = np.arctan2((P - cen) @ e2, (P - cen) @ e1)
    P = P[np.argsort(ang)]
    total = 0.0
    for i in range(len(P)):
        A, B = P[i], P[(i + 1) % len(P)]
        area = 0.5 * float(np.linalg.norm(np.cross(A - cen, B - cen)))
        # map the reference triangle to (cen, A, B): collapsed Gauss in 2D
        gx, gw = gauss_legendre(5)
        for (s, ws), (t, wt) in itertools.product(zip(gx, gw), repeat=2):
            x = cen + s * (A - cen) + (1 - s) * t * (B - cen)
            total += ws * wt * (1 - s) * 2 * area * float(np.prod(x ** np.array(alpha)))
    return total


def _alphas(d, deg):
    return [a for a in itertools.product(range(deg + 1), repeat=d) if sum(a) <= deg]


PLANES = [
    (3, np.array([0.3, -0.5, 0.81]), 0.07, 3),
    (3, np.array([1.0, 1.0, 1.0]), 0.31, 2),
    (3, np.array([0.0, 0.2, 1.0]), -0.03, 4),
    (3, np.array([0.0, 0.0, 1.0]), 0.011, 3),
    (2, np.array([0.6, -0.8]), 0.05, 3),
    (2, np.array([1.0, 0.0]), -0.02, 4),
]


def _cut_boxes(pl, d, h=0.25, limit=6):
    """boxes of a small grid around the origin that the plane cuts"""
    out = []
    for ijk in itertools.product(range(-2, 2), repeat=d):
        lo = np.array(ijk, dtype=float) * h
        hi = lo + h
        if box_class(pl, lo, hi) == CUT:
            out.append((lo, hi))
    return out[:limit]


@pytest.mark.parametrize("d,nrm,off,q", PLANES)
def test_plane_cell_rules_have_exact_moments(d, nrm, off, q):
    pl = Plane(nrm, off)
    S = SayeQuadrature(pl, d, q)
    boxes = _cut_boxes(pl, d)
    assert boxes
    for lo, hi in boxes:
        vx, vw, sx, sw, sn = S.cell_rule(lo, hi)
        vx, sx, sn = vx.reshape(-1, d), sx.reshape(-1, d), sn.reshape(-1, d)
        P = _clip_box(lo, hi, pl.n, pl.c0)
        for alpha in _alphas(d, 2 * q - d):
            ref = _polytope_moment(P, alpha)
            got = float(np.sum(vw * np.prod(vx ** np.array(alpha), axis=1)))
            assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref)) + 1e-16, (alpha, got, ref)
        for alpha in _alphas(d, 2 * q - d + 1):
            ref = _section_moment(lo, hi, pl.n, pl.c0, alpha)
            got = float(np.sum(sw * np.prod(sx ** np.array(alpha), axis=1)))
            assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref)) + 1e-16, ("surface", alpha, got, ref)
        assert np.allclose(sn, pl.n[None, :], rtol=0, atol=1e-15)
        assert (vw > 0).all() and (sw > 0).all()


@pytest.mark.parametrize("d,nrm,off,q", [p for p in PLANES if p[0] == 3])
def test_plane_face_rules_have_exact_moments(d, nrm, off, q):
    """cut faces: the rule on {phi < 0} of a face x_axis = const of a cut box
    against the moments of the clipped square (in-face coordinates)."""
    pl = Plane(nrm, off)
    S = SayeQuadrature(pl, d, q)
    n_checked = 0
    for lo, hi in _cut_boxes(pl, d, limit=20):
        for axis in range(3):
            value = hi[axis]
            flo, fhi = lo.copy(), hi.copy()
            flo[axis] = fhi[axis] = value
            fmn, fmx = pl.box_range(flo, fhi)
            if not (fmn < 0.0 < fmx):
                continue
            fx, fw = S.face_rule(lo, hi, axis, value)
            other = [a for a in range(3) if a != axis]
            n2 = pl.n[other]
            c2 = pl.c0 - pl.n[axis] * value
            if np.all(n2 == 0):
                continue
            P = _clip_box(lo[other], hi[other], n2, c2)
            for alpha in _alphas(2, 2 * q - 2):
                ref = _polytope_moment(P, alpha)
                got = float(np.sum(fw * np.prod(fx[:, other] ** np.array(alpha), axis=1)))
                assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref)) + 1e-16, (axis, alpha, got, ref)
            n_checked += 1
    assert n_checked > 0


def test_plane_classification_matches_corner_signs():
    """inside iff phi < 0 at every corner, outside iff phi >= 0 at every
    corner (the plane is linear, so its extremes over a box are at corners)"""
    mesh = Mesh(3, 9)
    pl = Plane([0.2, -0.4, 0.9], 0.13)
    cls = classify_cells(mesh, pl)
    for b in range(mesh.n_cells):
        lo, hi = mesh.cell_box(b)
        vals = [pl.phi(np.array([hi[a] if (k >> a) & 1 else lo[a] for a in range(3)])) for k in range(8)]
        expect = INSIDE if max(vals) < 0 else (OUTSIDE if min(vals) >= 0 else CUT)
        assert cls[b] == expect == box_class(pl, lo, hi), b


def test_moment_reference_catches_a_wrong_rule():
    """the reference sees a wrong interface weight (|n_k| dropped) and a
    shifted plane"""
    pl = Plane([0.3, -0.5, 0.81], 0.07)
    S = SayeQuadrature(pl, 3, 3)
    lo, hi = _cut_boxes(pl, 3)[0]
    vx, vw, sx, sw, sn = S.cell_rule(lo, hi)
    area = _section_moment(lo, hi, pl.n, pl.c0, (0, 0, 0))
    k = int(np.argmax(np.abs(pl.n)))
    assert abs(float(np.sum(sw)) - area) < 1e-13
    assert abs(float(np.sum(sw * abs(pl.n[k]))) - area) > 1e-3 * area
    vol = _polytope_moment(_clip_box(lo, hi, pl.n, pl.c0 + 1e-3), (0, 0, 0))
    assert abs(float(np.sum(vw)) - vol) > 1e-6


@pytest.mark.parametrize("dim,n,p,nrm,off", [(3, 8, 2, [0.3, -0.5, 0.81], 0.07), (2, 10, 3, [0.6, -0.8], 0.05)])
def test_operator_closed_forms_for_linear_u_below_a_plane(dim, n, p, nrm, off):
    """u = a . x + beta below a plane through the box.  SIPG and ghost
    penalty vanish for a continuous linear u, and the background box
    boundary carries no term, so with the Nitsche terms (Section 2.1)
      1^T A u = -(a . n)|Gamma| + (tau/h) (a . int_Gamma x + beta |Gamma|),
      u^T A u = |a|^2 |Omega| - 2 (a . n) int_Gamma u + (tau/h) int_Gamma u^2,
    with |Omega| and the moments over Gamma from the clipped polytopes."""
    from oracle.operator import UnfittedDG

    op = UnfittedDG(dim, n, p, np.zeros((0, dim)), np.zeros(0), plane=(np.array(nrm), off))
    pl = op.balls
    a = np.array([0.4, -0.7, 0.25][:dim])
    beta = 0.3
    u = op.dof_values_of(lambda x: float(a @ x) + beta)
    Au = op.apply(u)
    lo, hi = -np.ones(dim), np.ones(dim)
    vol = _polytope_moment(_clip_box(lo, hi, pl.n, pl.c0), (0,) * dim)
    e = np.eye(dim, dtype=int)
    G0 = _section_moment(lo, hi, pl.n, pl.c0, (0,) * dim)
    G1 = np.array([_section_moment(lo, hi, pl.n, pl.c0, tuple(e[i])) for i in range(dim)])
    G2 = np.array([[_section_moment(lo, hi, pl.n, pl.c0, tuple(e[i] + e[j])) for j in range(dim)] for i in range(dim)])
    an = float(a @ pl.n)
    int_u = float(a @ G1) + beta * G0
    int_u2 = float(a @ G2 @ a) + 2 * beta * float(a @ G1) + beta**2 * G0
    t = op.tau / op.h
    one_Au = -an * G0 + t * int_u
    uAu = float(a @ a) * vol - 2 * an * int_u + t * int_u2
    assert abs(Au.sum() - one_Au) <= 1e-11 * (abs(one_Au) + t * G0)
    assert abs(u @ Au - uAu) <= 1e-11 * (abs(uAu) + t * G0)
    # a wrong sign of the normal or a dropped Nitsche term would show
    assert abs(uAu - (float(a @ a) * vol + 2 * an * int_u + t * int_u2)) > 1e-6
