"""Pins of the oracle's volume ghost penalty (Section 2.2, eq.
volume_based_gp; evaluation by shifted Gauss points as in Section 3.3):

* it vanishes for every polynomial of degree <= p (one polynomial across a
  patch has no jump),
* the indicator of one cell has u^T G u = 2 tau_v h^(d-2) per patch of that
  cell (the jump is 1 on both halves of the patch),
* the coupling of a patch is the Kronecker product of 1D matrices integrated
  exactly with numpy polynomials over the two-cell patch (no quadrature),
* symmetry and positive semi-definiteness,
* the stable-neighbour patches pair every cut cell with a neighbour of
  largest volume fraction.
"""
import math

import numpy as np
import numpy.polynomial.polynomial as P
import pytest

import ufem_inputs as ui
from oracle.basis import gauss_lobatto_nodes
from oracle.geometry import CUT, INSIDE, OUTSIDE
from oracle.operator import GP, UnfittedDG


def _op(dim=3, n=8, p=2, seed=1, kind="volume", tau=0.1):
    wl, rng = (ui.ball3d(seed, n=n, degree=p) if dim == 3 else ui.disk2d(seed, n=n, degree=p))
    return UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, gp_kind=kind, gp_gamma=tau), rng


@pytest.fixture(scope="module")
def ball():
    return _op()


@pytest.fixture(scope="module")
def disk():
    return _op(dim=2, n=12, p=3, seed=2)


@pytest.mark.parametrize("which", ["ball", "disk"])
def test_vanishes_for_polynomials_of_degree_p(which, ball, disk):
    op, _ = ball if which == "ball" else disk
    p = op.p
    rng = np.random.default_rng(3)
    c = rng.uniform(-1, 1, (p + 1,) * op.dim)

    def f(x):
        val = 0.0
        for idx in np.ndindex(*c.shape):
            if sum(idx) <= p:
                val += c[idx] * np.prod([x[a] ** idx[a] for a in range(op.dim)])
        return val

    u = op.dof_values_of(f)
    g = op.apply(u, GP)
    scale = op.tau_v * op.h ** (op.dim - 2) * np.abs(u).max()
    assert np.abs(g).max() < 1e-11 * scale
    # while a discontinuous field is penalised
    u2 = u.copy()
    u2[: op.nd] += 1.0
    assert np.abs(op.apply(u2, GP)).max() > 0.1 * scale / np.abs(u).max()


@pytest.mark.parametrize("which", ["ball", "disk"])
def test_cell_indicator(which, ball, disk):
    op, _ = ball if which == "ball" else disk
    patches = [f for f in op.faces if f[4]]
    assert patches
    for b in (op.cut_cells[0], op.cut_cells[len(op.cut_cells) // 2], op.inside_cells[0]):
        u = np.zeros(op.n_dofs)
        r = op.rank[b]
        u[r * op.nd:(r + 1) * op.nd] = 1.0
        n_p = sum(1 for f in patches if b in (f[0], f[1]))
        val = u @ op.apply(u, GP)
        assert abs(val - 2 * op.tau_v * op.h ** (op.dim - 2) * n_p) < 1e-12 * max(1.0, val)


def _exact_patch_1d(p):
    """1D GLL basis on [0, 1]; the own cell at [0, 1] and its neighbour at
    [1, 2] (s = 1) or at [-1, 0] (s = 0): exact integrals over the patch of
    phi_i phi_j (own-own) and phi_i phi_j(x -+ 1) (own-neighbour)."""
    x = gauss_lobatto_nodes(p + 1)
    L = []
    for i in range(p + 1):
        roots = [x[j] for j in range(p + 1) if j != i]
        cc = P.polyfromroots(roots) if roots else np.array([1.0])
        L.append(cc / P.polyval(x[i], cc))

    def shift(cc, t):  # c(x - t)
        out = np.zeros(1)
        for k, ck in enumerate(cc):
            out = P.polyadd(out, ck * P.polypow([-t, 1.0], k))
        return out

    def integ(cc, a, b):
        ci = P.polyint(cc)
        return P.polyval(b, ci) - P.polyval(a, ci)

    out = {}
    for s, (a, b, t) in {1: (0.0, 2.0, 1.0), 0: (-1.0, 1.0, -1.0)}.items():
        own = np.array([[integ(P.polymul(L[i], L[j]), a, b) for j in range(p + 1)] for i in range(p + 1)])
        cross = np.array([[integ(P.polymul(L[i], shift(L[j], t)), a, b) for j in range(p + 1)] for i in range(p + 1)])
        out[s] = (own, cross)
    M = np.array([[integ(P.polymul(L[i], L[j]), 0.0, 1.0) for j in range(p + 1)] for i in range(p + 1)])
    return out, M


def _kron(mats):
    out = np.array([[1.0]])
    for a in range(len(mats) - 1, -1, -1):
        out = np.kron(out, mats[a])
    return out


def test_patch_blocks_are_kronecker_products(ball):
    op, _ = ball
    ex, M = _exact_patch_1d(op.p)
    s = op.tau_v * op.h ** (op.dim - 2)
    fi = next(i for i, f in enumerate(op.faces) if f[4])
    bm, bp, a, _, _ = op.faces[fi]
    A = np.zeros((2 * op.nd, 2 * op.nd))
    # columns of the two cells' unit vectors through the GP term alone
    for col in range(2 * op.nd):
        u = np.zeros(op.n_dofs)
        cell = bm if col < op.nd else bp
        u[op.rank[cell] * op.nd + col % op.nd] = 1.0
        g = np.zeros(op.n_dofs)
        op._volume_gp(fi, op._block(u, bm), op._block(u, bp), g, {bm, bp})
        A[:op.nd, col] = op._block(g, bm)
        A[op.nd:, col] = op._block(g, bp)
    mats_own_lo = [ex[1][0] if ax == a else M for ax in range(op.dim)]
    mats_cross_lo = [ex[1][1] if ax == a else M for ax in range(op.dim)]
    mats_own_hi = [ex[0][0] if ax == a else M for ax in range(op.dim)]
    mats_cross_hi = [ex[0][1] if ax == a else M for ax in range(op.dim)]
    ref = np.block([[s * _kron(mats_own_lo), -s * _kron(mats_cross_lo)],
                    [-s * _kron(mats_cross_hi), s * _kron(mats_own_hi)]])
    assert np.abs(A - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("kind", ["volume", "volume_all"])
def test_symmetric_positive_semidefinite(kind):
    op, rng = _op(dim=2, n=8, p=2, seed=4, kind=kind)
    G = np.zeros((op.n_dofs, op.n_dofs))
    e = np.zeros(op.n_dofs)
    for j in range(op.n_dofs):
        e[j] = 1.0
        G[:, j] = op.apply(e, GP)
        e[j] = 0.0
    assert np.abs(G - G.T).max() < 1e-14 * np.abs(G).max()
    assert np.linalg.eigvalsh(G).min() > -1e-13 * np.abs(G).max()


def test_stable_neighbour_has_the_largest_volume_fraction(ball):
    op, _ = ball
    patches = [f for f in op.faces if f[4]]
    partner = {}
    for bm, bp, a, kind, gp in patches:
        partner.setdefault(bm, []).append(bp)
        partner.setdefault(bp, []).append(bm)
    for b in op.cut_cells:
        ijk = op.mesh.index_to_ijk(b)
        fr = []
        for a in range(op.dim):
            for side in (0, 1):
                if (side == 0 and ijk[a] == 0) or (side == 1 and ijk[a] == op.mesh.n - 1):
                    continue
                nb = b + (1 if side else -1) * op.mesh.strides[a]
                if op.cls[nb] != OUTSIDE:
                    fr.append((op.volume_fraction(nb), nb))
        best = max(f for f, _ in fr)
        chosen = [nb for nb in partner.get(b, []) if any(nb == x for _, x in fr)]
        assert any(abs(op.volume_fraction(nb) - best) <= 1e-10 for nb in chosen), b
    # the all-neighbours strategy keeps every face of a cut cell
    op_all, _ = _op(kind="volume_all")
    assert all(f[4] == (op_all.cls[f[0]] == CUT or op_all.cls[f[1]] == CUT) for f in op_all.faces)
