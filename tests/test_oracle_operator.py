"""Pins of the oracle operator against what the mathematics fixes:

* symmetry and positive definiteness,
* closed forms for linear and constant u on a disk / ball strictly inside the
  box (Section 2.1 forms; the divergence theorem gives the volume-Nitsche
  identity),
* consistency: for a polynomial u of degree <= p the SIPG and ghost-penalty
  jumps vanish and a(v, u) = -(v, Lap u) - (d_n v, u)_Gamma + tau/h (v, u)_Gamma,
* the Kronecker structure of the operator on uncut cells, built from 1D
  matrices integrated exactly with numpy polynomials (no quadrature),
* the ghost-penalty weights gamma_j h^(2j-1) on a derivative jump of order j,
* the SIPG penalty on piecewise constants,
* the coefficient derivative against central finite differences.
"""
import math

import numpy as np
import numpy.polynomial.polynomial as P
import pytest

import ufem_inputs as ui
from oracle.basis import gauss_lobatto_nodes
from oracle.geometry import CUT, INSIDE
from oracle.operator import ALL, GP, NITSCHE, SIPG, VOL, UnfittedDG


def disk_op(p=2, n=16, seed=0, q=None):
    wl, rng = ui.disk2d(seed, n=n, degree=p)
    return UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, q=q), wl, rng


def ball_op(p=2, n=8, R=0.8, seed=0, q=None):
    wl, rng = ui.ball3d(seed, n=n, degree=p, radius=R)
    return UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, q=q), wl, rng


@pytest.fixture(scope="module")
def disk():
    return disk_op()


@pytest.fixture(scope="module")
def ball():
    return ball_op()


@pytest.fixture(scope="module")
def disk_q6():
    return disk_op(q=6)


@pytest.fixture(scope="module")
def ball_q6():
    return ball_op(q=6)


def measures(wl):
    R = wl.radii[0]
    if wl.dim == 2:
        return math.pi * R**2, 2 * math.pi * R
    return 4 / 3 * math.pi * R**3, 4 * math.pi * R**2


@pytest.mark.parametrize("which", ["disk", "ball"])
def test_symmetry(which, disk, ball):
    op, wl, _ = disk if which == "disk" else ball
    rng = np.random.default_rng(11)
    u = rng.uniform(-1, 1, op.n_dofs)
    w = rng.uniform(-1, 1, op.n_dofs)
    for mask in (VOL, SIPG, NITSCHE, GP, ALL):
        a = w @ op.apply(u, mask)
        b = u @ op.apply(w, mask)
        assert abs(a - b) <= 1e-13 * (abs(a) + np.linalg.norm(op.apply(u, mask)) * np.linalg.norm(w))


def test_positive_definite_disk():
    op, wl, _ = disk_op(p=1, n=10)
    A = op.assemble()
    assert np.allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev[0] > 0.0


@pytest.mark.parametrize("which", ["disk", "ball"])
def test_linear_and_constant_closed_forms(which, disk, ball):
    op, wl, _ = disk if which == "disk" else ball
    d = wl.dim
    vol, area = measures(wl)
    R = wl.radii[0]
    c = wl.centers[0]
    a = np.array([0.3, -0.7, 0.45])[:d]
    beta = 0.4
    u = op.dof_values_of(lambda x: a @ x + beta)
    th = op.tau / op.h
    aa = a @ a
    alpha = a @ c + beta
    exact = -aa * vol + th * (aa * R**2 * area / d + alpha**2 * area)
    tol = 2e-5
    assert abs(u @ op.apply(u) / exact - 1) < tol
    assert abs(u @ op.apply(u, VOL) / (aa * vol) - 1) < tol
    assert abs(np.ones(op.n_dofs) @ op.apply(u) / (th * alpha * area) - 1) < tol
    # continuous u: every derivative jump vanishes, so the ghost penalty
    # gives nothing and the SIPG quadratic form vanishes
    scale = np.linalg.norm(op.apply(u))
    assert np.linalg.norm(op.apply(u, GP)) < 1e-12 * scale
    assert abs(u @ op.apply(u, SIPG)) < 1e-12 * scale * np.linalg.norm(u)
    uc = np.full(op.n_dofs, beta)
    assert abs(uc @ op.apply(uc) / (th * beta**2 * area) - 1) < tol


@pytest.mark.parametrize("which", ["disk", "ball"])
def test_consistency_for_polynomial_u(which, disk_q6, ball_q6):
    # a finer cut-cell rule (q = 6) brings the quadrature error of the
    # divergence theorem on cut cells below the tolerance
    op, wl, _ = disk_q6 if which == "disk" else ball_q6
    d = wl.dim
    if d == 2:
        f = lambda x: x[0] ** 2 - 0.5 * x[1] ** 2 + 0.3 * x[0] * x[1] + 0.2 * x[0]
        grad = lambda X: np.stack([2 * X[:, 0] + 0.3 * X[:, 1] + 0.2, -X[:, 1] + 0.3 * X[:, 0]], 1)
        lap = 2.0 - 1.0
    else:
        f = lambda x: x[0] ** 2 - 0.5 * x[1] ** 2 + 1.5 * x[2] ** 2 + 0.3 * x[0] * x[2] - 0.1 * x[1]
        grad = lambda X: np.stack(
            [2 * X[:, 0] + 0.3 * X[:, 2], -X[:, 1] - 0.1, 3 * X[:, 2] + 0.3 * X[:, 0]], 1
        )
        lap = 2.0 - 1.0 + 3.0
    u = op.dof_values_of(f)
    Au = op.apply(u)
    # right-hand side: -(v, Lap u)_Omega - (d_n v, u)_Gamma + tau/h (v, u)_Gamma
    b = np.zeros(op.n_dofs)
    h = op.h
    for cell in op.active:
        cell = int(cell)
        lo, _ = op.mesh.cell_box(cell)
        r = op.rank[cell]
        if op.cls[cell] == INSIDE:
            xi, w = op.full_cell_rule()
            xs = None
        else:
            xi, w, xs, ws, ns = op.cell_rule(cell)
        if xi.shape[0]:
            Phi = op.basis(xi)
            b[r * op.nd : (r + 1) * op.nd] += h**d * Phi.T @ (w * -lap)
        if xs is not None and xs.shape[0]:
            X = lo + h * xs
            uq = np.array([f(x) for x in X])
            Phi = op.basis(xs)
            dn = np.einsum("qla,qa->ql", op.grad_basis(xs), ns) / h
            b[r * op.nd : (r + 1) * op.nd] += h ** (d - 1) * (
                -dn.T @ (ws * uq) + (op.tau / h) * Phi.T @ (ws * uq)
            )
    assert np.linalg.norm(Au - b) < 1e-6 * np.linalg.norm(b)


def _exact_1d(p, gamma):
    """1D GLL Lagrange mass, stiffness and SIPG face matrices on [0, 1] by
    exact polynomial integration."""
    x = gauss_lobatto_nodes(p + 1)
    k = p + 1
    L = []
    for i in range(k):
        roots = [x[j] for j in range(k) if j != i]
        c = P.polyfromroots(roots) if roots else np.array([1.0])
        L.append(c / P.polyval(x[i], c))
    dL = [P.polyder(c) for c in L]

    def integ(c):
        ci = P.polyint(c)
        return P.polyval(1.0, ci) - P.polyval(0.0, ci)

    M = np.array([[integ(P.polymul(L[i], L[j])) for j in range(k)] for i in range(k)])
    K = np.array([[integ(P.polymul(dL[i], dL[j])) for j in range(k)] for i in range(k)])
    e0 = np.array([P.polyval(0.0, c) for c in L])
    e1 = np.array([P.polyval(1.0, c) for c in L])
    g0 = np.array([P.polyval(0.0, c) for c in dL])
    g1 = np.array([P.polyval(1.0, c) for c in dL])
    # face at xi = 1 (cell is the lower side) and at xi = 0 (upper side)
    F1 = -0.5 * np.outer(g1, e1) - 0.5 * np.outer(e1, g1) + gamma * np.outer(e1, e1)
    N1 = 0.5 * np.outer(g1, e0) - 0.5 * np.outer(e1, g0) - gamma * np.outer(e1, e0)
    F0 = 0.5 * np.outer(g0, e0) + 0.5 * np.outer(e0, g0) + gamma * np.outer(e0, e0)
    N0 = -0.5 * np.outer(g0, e1) + 0.5 * np.outer(e0, g1) - gamma * np.outer(e0, e1)
    return M, K, F1, N1, F0, N0


def _kron_dir(mats_by_axis):
    """Kronecker product with axis 0 fastest."""
    out = np.array([[1.0]])
    for a in range(len(mats_by_axis) - 1, -1, -1):
        out = np.kron(out, mats_by_axis[a])
    return out


@pytest.mark.parametrize("dim,p,n", [(2, 2, 8), (2, 3, 8), (3, 1, 8), (3, 3, 6)])
def test_kronecker_structure_on_uncut_cells(dim, p, n):
    centers = np.full((1, dim), 0.013)
    op = UnfittedDG(dim, n, p, centers, [0.93])
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, op.n_dofs)
    Au = op.apply(u)
    M, K, F1, N1, F0, N0 = _exact_1d(p, op.gamma)
    s = op.h ** (dim - 2)
    checked = 0
    for cell in op.inside_cells:
        ijk = op.mesh.index_to_ijk(cell)
        nbs = []
        ok = True
        for a in range(dim):
            for side in (-1, 1):
                if not (0 <= ijk[a] + side < n):
                    ok = False
                    continue
                nb = cell + side * op.mesh.strides[a]
                if op.cls[nb] != INSIDE:
                    ok = False
                nbs.append((a, side, nb))
        if not ok:
            continue
        own = np.zeros((op.nd, op.nd))
        for a in range(dim):
            mats = [M] * dim
            mats = list(mats)
            mats[a] = K + F1 + F0
            own += _kron_dir(mats)
        v = own @ op._block(u, cell)
        for a, side, nb in nbs:
            mats = [M] * dim
            mats = list(mats)
            mats[a] = N1 if side == 1 else N0
            v += _kron_dir(mats) @ op._block(u, nb)
        v *= s
        assert np.allclose(op._block(Au, cell), v, rtol=0, atol=1e-12 * np.abs(v).max())
        checked += 1
    assert checked > 0


@pytest.mark.parametrize("j", [0, 1, 2])
def test_ghost_penalty_weight_of_order_j(j):
    """u = (x - x_F)^j on the cells right of a mesh plane x = x_F, 0 on the
    left: only the j-th derivative jumps (by -j!) on that plane, so
    u^T A_gp u = gamma_j h^(2j-1) (j!)^2 |F| per ghost-penalty face."""
    op, wl, _ = disk_op(p=2, n=16)
    xF = op.mesh.lo + 8 * op.h
    u = op.dof_values_of(lambda x: (x[0] - xF) ** j if x[0] > xF - 1e-12 else 0.0)
    # the left cells' DoFs on the plane belong to the left cell: zero them
    for cell in op.active:
        ijk = op.mesh.index_to_ijk(int(cell))
        if ijk[0] < 8:
            op._block(u, int(cell))[:] = 0.0
    n_gp = sum(
        1 for (bm, bp, a, kind, gp) in op.faces if gp and a == 0 and op.mesh.index_to_ijk(bm)[0] == 7
    )
    assert n_gp > 0
    exact = op.gp_w[j] * op.h ** (2 * j - 1) * math.factorial(j) ** 2 * op.h ** (wl.dim - 1) * n_gp
    assert abs(u @ op.apply(u, GP) / exact - 1) < 1e-12


def test_sipg_penalty_on_piecewise_constants(disk):
    op, wl, _ = disk
    rng = np.random.default_rng(2)
    cvals = rng.uniform(-1, 1, op.active.size)
    u = np.repeat(cvals, op.nd)
    exact = 0.0
    for fi, (bm, bp, a, kind, gp) in enumerate(op.faces):
        if kind == "none":
            continue
        meas = op.face_rule(fi)[1].sum()
        exact += op.gamma * op.h ** (wl.dim - 2) * meas * (cvals[op.rank[bm]] - cvals[op.rank[bp]]) ** 2
    assert abs(u @ op.apply(u, SIPG) / exact - 1) < 1e-12


def test_dkappa_against_central_differences():
    wl, rng = ui.disk2d(0, n=10, degree=2)
    op = UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii)
    u = ui.uniform_vector(rng, op.n_dofs)
    b = ui.uniform_vector(rng, op.n_dofs)
    kap = ui.kappa_field(op.qp_physical_points())
    delta = rng.uniform(-1, 1, kap.size)

    def loss(k):
        r = op.apply(u, ALL, k) - b
        return 0.5 * r @ r

    r = op.apply(u, ALL, kap) - b
    g = op.dkappa(r, u)
    eps = 1e-6
    fd = (loss(kap + eps * delta) - loss(kap - eps * delta)) / (2 * eps)
    assert abs(fd - g @ delta) < 1e-7 * abs(fd) + 1e-9
    # with kappa == 1 the kappa-weighted terms reproduce the operator minus
    # the ghost penalty: sum_q dkappa_q(w, u) = w^T (A - A_gp) u
    w = ui.uniform_vector(rng, op.n_dofs)
    gq = op.dkappa(w, u)
    assert abs(gq.sum() - w @ (op.apply(u) - op.apply(u, GP))) < 1e-11 * abs(gq.sum())
