"""Pins of the oracle's continuous space (FE_Q, Section 2.1, eq.
bilinear_cg, with the ghost penalty of Section 2.2):

* closed forms for linear and constant u on a disk / ball strictly inside
  the box (Poisson and Nitsche terms; the ghost penalty vanishes on
  continuous polynomials of degree <= p): u^T A u = |a|^2 |Omega| -
  2 (a.n, u)_Gamma + tau/h (u, u)_Gamma with the divergence theorem, and
  1^T A u = tau/h (a.c + beta) |Gamma|,
* the SIPG term of the cell-DoF operator vanishes between continuous
  functions (so P^T A_cell P is the same with or without it),
* rows of nodes away from the cut equal the Kronecker sum of globally
  assembled 1D GLL stiffness and mass matrices integrated exactly with numpy
  polynomials (checks the node lattice, P and P^T),
* symmetry and positive definiteness.
"""
import math

import numpy as np
import numpy.polynomial.polynomial as Pn
import pytest

import ufem_inputs as ui
from oracle.basis import gauss_lobatto_nodes
from oracle.geometry import INSIDE
from oracle.operator import ALL, GP, NITSCHE, SIPG, VOL, UnfittedCG


def _cg(dim, n, p, seed, q=None):
    wl, rng = ui.disk2d(seed, n=n, degree=p) if dim == 2 else ui.ball3d(seed, n=n, degree=p)
    return UnfittedCG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, q=q), wl


@pytest.fixture(scope="module")
def disk():
    return _cg(2, 12, 3, 0, q=6)


@pytest.fixture(scope="module")
def ball():
    return _cg(3, 8, 2, 1, q=6)


@pytest.mark.parametrize("which", ["disk", "ball"])
def test_linear_and_constant_closed_forms(which, disk, ball):
    op, wl = disk if which == "disk" else ball
    d = wl.dim
    R = wl.radii[0]
    c = wl.centers[0]
    vol = math.pi * R**2 if d == 2 else 4 / 3 * math.pi * R**3
    area = 2 * math.pi * R if d == 2 else 4 * math.pi * R**2
    a = np.array([0.7, -0.4, 0.3][:d])
    beta = 0.25
    u = op.dof_values_of(lambda x: float(a @ x) + beta)
    Au = op.apply(u)
    t = op.dg.tau / op.h
    # (u, u)_Gamma and (a.n, u)_Gamma on the sphere |x - c| = R:
    # u = a.(x - c) + (a.c + beta); mean of (a.(x-c))^2 over the sphere is |a|^2 R^2 / d
    m = float(a @ c) + beta
    int_u2 = (float(a @ a) * R**2 / d + m * m) * area
    int_anu = float(a @ a) * R / d * area  # a.n = a.(x - c)/R, times u, integrated
    uAu = float(a @ a) * vol - 2 * int_anu + t * int_u2
    assert abs(u @ Au - uAu) < 2e-6 * abs(uAu)
    assert abs(Au.sum() - t * m * area) < 2e-6 * t * abs(m) * area
    ones = np.ones(op.n_dofs)
    assert abs(ones @ op.apply(ones) - t * area) < 2e-6 * t * area
    # the ghost penalty of a continuous polynomial of degree <= p vanishes
    assert np.abs(op.apply(u, GP)).max() < 1e-9 * np.abs(Au).max()


def test_sipg_vanishes_between_continuous_functions(ball):
    op, _ = ball
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, op.n_dofs)
    w = rng.uniform(-1, 1, op.n_dofs)
    s = op.gather(w) @ op.dg.apply(op.gather(u), SIPG)
    ref = abs(op.gather(w) @ op.dg.apply(op.gather(u), VOL))
    assert abs(s) < 1e-12 * ref


def _exact_1d(p):
    x = gauss_lobatto_nodes(p + 1)
    L = []
    for i in range(p + 1):
        roots = [x[j] for j in range(p + 1) if j != i]
        cc = Pn.polyfromroots(roots) if roots else np.array([1.0])
        L.append(cc / Pn.polyval(x[i], cc))
    dL = [Pn.polyder(c) for c in L]

    def integ(c):
        ci = Pn.polyint(c)
        return Pn.polyval(1.0, ci) - Pn.polyval(0.0, ci)

    M = np.array([[integ(Pn.polymul(L[i], L[j])) for j in range(p + 1)] for i in range(p + 1)])
    K = np.array([[integ(Pn.polymul(dL[i], dL[j])) for j in range(p + 1)] for i in range(p + 1)])
    return M, K


@pytest.mark.parametrize("dim,n,p", [(2, 10, 3), (3, 12, 2)])
def test_interior_rows_are_assembled_kronecker_sums(dim, n, p):
    wl, _ = ui.disk2d(3, n=n, degree=p) if dim == 2 else ui.ball3d(3, n=n, degree=p)
    op = UnfittedCG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii)
    M, K = _exact_1d(p)
    L1 = op.L1
    # globally assembled 1D matrices on the node line (cell size 1 in
    # reference units; h^(d-2) applied below)
    Mg = np.zeros((L1, L1))
    Kg = np.zeros((L1, L1))
    for c in range(n):
        sl = slice(c * p, c * p + p + 1)
        Mg[sl, sl] += M
        Kg[sl, sl] += K
    # nodes whose surrounding cells are inside cells with no ghost-penalty
    # face: every cell touching a node within two cells of it is inside
    dg = op.dg
    lat = op.lattice
    checked = 0
    rng = np.random.default_rng(0)
    for idx in rng.permutation(op.n_dofs):
        I = [(lat[idx] // L1**a) % L1 for a in range(dim)]
        cells = [range(max(0, i // p - 2), min(n, i // p + 2)) for i in I]
        box = np.stack(np.meshgrid(*cells, indexing="ij"), -1).reshape(-1, dim)
        if not all(dg.cls[int(sum(b[a] * n**a for a in range(dim)))] == INSIDE for b in box):
            continue
        e = np.zeros(op.n_dofs)
        e[idx] = 1.0
        row = op.apply(e, VOL)  # symmetric: the column equals the row
        # Kronecker sum on the full lattice, restricted to active nodes
        ref = np.zeros(L1**dim)
        for a in range(dim):
            vec = np.ones(1)
            for b in range(dim - 1, -1, -1):
                m = Kg if b == a else Mg
                vec = np.kron(vec, m[I[b]])
            ref += vec
        ref *= op.h ** (dim - 2)
        assert np.abs(row - ref[lat]).max() < 1e-13 * np.abs(ref).max()
        checked += 1
        if checked >= 4:
            break
    assert checked > 0


def test_symmetric_positive_definite():
    op, _ = _cg(2, 8, 2, 4)
    A = np.zeros((op.n_dofs, op.n_dofs))
    e = np.zeros(op.n_dofs)
    for j in range(op.n_dofs):
        e[j] = 1.0
        A[:, j] = op.apply(e)
        e[j] = 0.0
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0
