"""Pins of the oracle's classification and dimension-reduction quadrature
against closed forms: volume, area and moments of balls and of a union of two
balls, the divergence theorem cut cell by cut cell, and brute-force sampling
of the cell classes."""
import math

import numpy as np
import pytest

from oracle.geometry import CUT, INSIDE, OUTSIDE, Balls, Mesh, box_class, classify_cells
from oracle.quadrature import SayeQuadrature


def _integrate(dim, n, centers, radii, q, f_vol=None, f_surf=None):
    mesh = Mesh(dim, n)
    balls = Balls(np.array(centers), np.array(radii))
    cls = classify_cells(mesh, balls)
    sq = SayeQuadrature(balls, dim, q)
    gx = np.array(sq.gx)
    gw = np.array(sq.gw)
    vol = 0.0
    surf = 0.0
    for b in range(mesh.n_cells):
        lo, hi = mesh.cell_box(b)
        if cls[b] == INSIDE:
            # tensor Gauss on the cell
            grids = np.meshgrid(*[lo[a] + mesh.h * gx for a in range(dim)], indexing="ij")
            pts = np.stack([g.ravel() for g in grids], axis=1)
            wts = np.prod(np.stack(np.meshgrid(*[mesh.h * gw] * dim, indexing="ij")), axis=0).ravel()
            vol += np.sum(wts * (f_vol(pts) if f_vol else 1.0))
        elif cls[b] == CUT:
            vp, vw, sp, sw, sn = sq.cell_rule(lo, hi)
            if vw.size:
                vol += np.sum(vw * (f_vol(vp) if f_vol else 1.0))
            if sw.size:
                surf += np.sum(sw * (f_surf(sp, sn) if f_surf else 1.0))
    return vol, surf, sq


@pytest.mark.parametrize("dim", [2, 3])
def test_ball_measure_converges_with_q(dim):
    c = [0.013, -0.021, 0.017][:dim]
    R = 0.7
    exact_v = math.pi * R**2 if dim == 2 else 4.0 / 3.0 * math.pi * R**3
    exact_s = 2 * math.pi * R if dim == 2 else 4.0 * math.pi * R**2
    n = 16 if dim == 2 else 8
    errs = []
    for q in (2, 3, 4, 5):
        v, s, sq = _integrate(dim, n, [c], [R], q)
        errs.append((abs(v - exact_v) / exact_v, abs(s - exact_s) / exact_s))
        assert sq.n_fallback == 0
    for (ev0, es0), (ev1, es1) in zip(errs[:-1], errs[1:]):
        assert ev1 < 0.2 * ev0 and es1 < 0.2 * es0
    assert errs[-1][0] < 5e-8 and errs[-1][1] < 5e-7


def test_ball_moments_and_normals():
    c = np.array([0.02, -0.01, 0.03])
    R = 0.8
    q = 5
    # int_Omega (x - c) = 0 ; int_Omega |x - c|^2 = 4 pi R^5 / 5
    v1, _, _ = _integrate(3, 8, [c], [R], q, f_vol=lambda X: X[:, 0] - c[0])
    v2, _, _ = _integrate(3, 8, [c], [R], q, f_vol=lambda X: np.sum((X - c) ** 2, axis=1))
    assert abs(v1) < 1e-9
    assert abs(v2 / (4 * math.pi * R**5 / 5) - 1) < 1e-8
    # int_Gamma n = 0 ; int_Gamma (x - c).n = R |Gamma| (normals point out of Omega)
    _, s1, _ = _integrate(3, 8, [c], [R], q, f_surf=lambda X, N: N[:, 2])
    _, s2, _ = _integrate(3, 8, [c], [R], q, f_surf=lambda X, N: np.sum((X - c) * N, axis=1))
    assert abs(s1) < 1e-8
    assert abs(s2 / (R * 4 * math.pi * R**2) - 1) < 1e-7


def test_union_of_two_balls_volume_and_area():
    c1 = np.array([-0.21, 0.013, 0.02])
    c2 = np.array([0.24, -0.017, -0.011])
    R1, R2 = 0.5, 0.42
    d = float(np.linalg.norm(c2 - c1))
    lens = math.pi * (R1 + R2 - d) ** 2 * (d * d + 2 * d * (R1 + R2) - 3 * (R1 - R2) ** 2) / (12 * d)
    exact_v = 4 / 3 * math.pi * (R1**3 + R2**3) - lens
    x1 = (d * d + R1 * R1 - R2 * R2) / (2 * d)
    x2 = d - x1
    exact_s = 4 * math.pi * R1**2 - 2 * math.pi * R1 * (R1 - x1) + 4 * math.pi * R2**2 - 2 * math.pi * R2 * (R2 - x2)
    v, s, _ = _integrate(3, 12, [c1, c2], [R1, R2], 4)
    # the intersection curve of the two spheres is not a splitting set of the
    # lower-dimensional problems, so the integrand is only piecewise smooth
    # there and the rule converges at low order near it
    assert abs(v / exact_v - 1) < 2e-5
    assert abs(s / exact_s - 1) < 2e-3


def _face_rule_of_box_face(sq, balls, lo, hi, axis, value):
    flo = lo.copy()
    fhi = hi.copy()
    flo[axis] = value
    fhi[axis] = value
    return sq.face_rule(lo, hi, axis, value)


@pytest.mark.parametrize("dim,centers,radii,tol", [
    (2, [[0.013, -0.021]], [0.7], 1e-3),
    (3, [[0.01, 0.02, -0.03]], [0.8], 1e-3),
    # cells crossed by the intersection curve of two spheres: low order there
    (3, [[-0.2, 0.01, 0.0], [0.25, -0.02, 0.03]], [0.5, 0.45], 3e-2),
])
def test_divergence_theorem_on_every_cut_cell(dim, centers, radii, tol):
    """int_{T cap Omega} div F = int_{Gamma cap T} F.n + int_{dT cap Omega} F.n_T
    for a polynomial field F: ties the volume, interface and face rules and
    the normal orientation together.  A wrong sign, weight or orientation
    gives an O(1) relative defect; the bound leaves room for the slow
    convergence of the height-function rule near nearly tangent cuts."""
    mesh = Mesh(dim, 8)
    balls = Balls(np.array(centers), np.array(radii))
    cls = classify_cells(mesh, balls)
    sq = SayeQuadrature(balls, dim, 5)
    A = np.array([[0.3, -1.1, 0.7], [0.5, 0.2, -0.4], [-0.6, 0.9, 0.1]])[:dim, :dim]

    def F(X):
        # F_a = sum_b A_ab x_b^2 + x_a x_{a+1}
        out = (X**2) @ A.T
        out += X * np.roll(X, -1, axis=1)
        return out

    def divF(X):
        return np.sum(2 * np.diag(A)[None, :] * X + np.roll(X, -1, axis=1), axis=1)

    worst = 0.0
    for b in np.nonzero(cls == CUT)[0]:
        lo, hi = mesh.cell_box(int(b))
        vp, vw, sp, sw, sn = sq.cell_rule(lo, hi)
        lhs = np.sum(vw * divF(vp)) if vw.size else 0.0
        rhs = np.sum(sw * np.sum(F(sp) * sn, axis=1)) if sw.size else 0.0
        for a in range(dim):
            for side, val in ((-1.0, lo[a]), (1.0, hi[a])):
                pts, w = sq.face_rule(lo, hi, a, val)
                if w.size:
                    rhs += side * np.sum(w * F(pts)[:, a])
        worst = max(worst, abs(lhs - rhs) / mesh.h ** (dim - 1))
    assert worst < tol


@pytest.mark.parametrize("dim,centers,radii", [
    (2, [[0.013, -0.021]], [0.7]),
    (3, [[0.2, -0.1, 0.05], [-0.3, 0.2, 0.1]], [0.35, 0.3]),
])
def test_classification_against_sampling(dim, centers, radii):
    mesh = Mesh(dim, 10)
    balls = Balls(np.array(centers), np.array(radii))
    cls = classify_cells(mesh, balls)
    rng = np.random.default_rng(3)
    s = rng.uniform(0.0, 1.0, size=(400, dim))
    s = np.concatenate([s, np.array(np.meshgrid(*[[0.0, 1.0]] * dim)).reshape(dim, -1).T])
    n_cut_seen = 0
    for b in range(mesh.n_cells):
        lo, hi = mesh.cell_box(b)
        assert box_class(balls, lo, hi) == cls[b]
        phi = balls.phi_many(lo + mesh.h * s)
        if cls[b] == INSIDE:
            assert np.all(phi < 0)
        elif cls[b] == OUTSIDE:
            assert np.all(phi >= 0)
        else:
            n_cut_seen += 1
            assert np.any(phi > 0) or np.all(phi < 0)  # cut or jointly covered
    assert n_cut_seen > 0
