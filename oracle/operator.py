"""The unfitted DG (SIPG) Poisson operator v = A u, evaluated naively.

Test infrastructure only (see the package docstring).

Discrete form (Section 2.1, bilinear forms of the CG and DG methods; Section
2.2 for the stabilisation), with a coefficient kappa that is 1 unless given:

  a(v, u) =   (kappa grad v, grad u)_{Omega}                          volume
            - (kappa d_n v, u)_Gamma - (v, kappa d_n u)_Gamma
            + (tau_D / h) (kappa v, u)_Gamma                          Nitsche
            - ({kappa d_n v}, [u])_F - ([v], {kappa d_n u})_F
            + (gamma / h) (kappa [v], [u])_F      over F cap Omega     SIPG
            + sum_j gamma_j h^(2j-1) ([d_n^j v], [d_n^j u])_F  full F  ghost penalty

with [w] = w^- - w^+, {w} = (w^- + w^+)/2, n = +e_axis on a face between the
lower (-) and upper (+) cell, tau_D = nitsche_factor p^2,
gamma = sipg_factor p^2, gamma_j = gp_gamma / (j!)^2 (or gp_gamma for every j
with gp_weights='flat'), j = gp_jmin..p.

The face ghost penalty is only referred to (its treatment lives in a
supplement that is not part of the text); the form above is the standard face
ghost penalty of Burman (2010), with the weights as stated.

With gp_kind='volume' the ghost penalty is instead the volume-based one of
Section 2.2 (eq. volume_based_gp), the paper's own choice:

  g_v(v, u) = sum over patches P of (tau_v / h^2) (J_P v, J_P u)_P,

a patch being two face neighbours E1, E2 and J_P u the difference of the two
cells' polynomials, each extended to the whole patch (u1 - E u2 on E1 and
E u1 - u2 on E2, E the extension of a cell's polynomial to its neighbour).
As in Section 3.3 the extension is evaluated by shifting the Gauss points of
one cell into the reference coordinates of the other (values of the Lagrange
basis outside [0, 1]), and the integrals use the k^d Gauss rule of each
whole cell.  Patches (stable-neighbour strategy of Section 2.2): every cut
cell is paired with the face neighbour of largest volume fraction |N cap
Omega| / |N| (1 for inside cells; for cut cells the sum of the reference
weights of their volume rule), fractions within 1e-10 counting as equal and
the lower slot 2 axis + side winning; a patch chosen by both of its cells
counts once.  gp_kind='volume_all' takes every face of a cut cell instead
(all-neighbours strategy).  tau_v is gp_gamma.

Every term is evaluated on the reference cell [0, 1]^d: with x = x_0 + h xi
every term scales with h^(d-2) (gradients carry 1/h, volumes h^d, faces and
the interface h^(d-1), penalties 1/h, the j-th ghost-penalty derivative
h^-j).  Basis functions are evaluated at each quadrature point with the full
tensor product (naive evaluation, Section 3.2), no sum factorisation.

DoF layout: cell-contiguous, active cells in background order, local index
l = i + k j + k^2 m (x fastest, Section 3.2).

Quadrature-point (kappa) layout, one segment after the other:
  [ volume of inside cells (k^d Gauss points each, active order)
  | volume of cut cells (dimension-reduction points, active order)
  | structured SIPG faces (k^(d-1) Gauss points each, face order)
  | cut SIPG faces (dimension-reduction points, face order)
  | interface points of cut cells (active order) ]
"""
from __future__ import annotations

import math

import numpy as np

from .basis import gauss_legendre, gauss_lobatto_nodes, lagrange_derivatives
from .geometry import CUT, INSIDE, OUTSIDE, Balls, Mesh, Plane, active_faces, classify_cells
from .quadrature import SayeQuadrature

VOL, SIPG, NITSCHE, GP = 1, 2, 4, 8
ALL = VOL | SIPG | NITSCHE | GP


def _tensor_product(vals):
    """vals[a] is (nq, k); returns (nq, k^d) with axis 0 fastest."""
    nq = vals[0].shape[0]
    F = np.ones((nq, 1))
    for a in range(len(vals) - 1, -1, -1):
        F = (F[:, :, None] * vals[a][:, None, :]).reshape(nq, -1)
    return F


class UnfittedDG:
    def __init__(
        self,
        dim,
        n,
        degree,
        centers,
        radii,
        lo=-1.0,
        hi=1.0,
        q=None,
        max_depth=4,
        nitsche_factor=20.0,
        sipg_factor=20.0,
        gp_gamma=0.1,
        gp_jmin=0,
        gp_weights="factorial",
        plane=None,
        gp_kind="face",
    ):
        self.dim = dim
        self.p = degree
        self.k = degree + 1
        self.nd = self.k**dim
        self.mesh = Mesh(dim, n, lo, hi)
        self.h = self.mesh.h
        # level set: a union of balls, or with plane = (normal, offset) the
        # half space n . x < offset of the plane benchmark
        self.balls = Balls(centers, radii) if plane is None else Plane(plane[0], plane[1])
        self.q = self.k if q is None else q
        self.saye = SayeQuadrature(self.balls, dim, self.q, max_depth)
        self.tau = nitsche_factor * degree**2
        self.gamma = sipg_factor * degree**2
        self.gp_j = list(range(gp_jmin, degree + 1))
        if gp_weights == "factorial":
            self.gp_w = {j: gp_gamma / math.factorial(j) ** 2 for j in self.gp_j}
        elif gp_weights == "flat":
            self.gp_w = {j: gp_gamma for j in self.gp_j}
        else:
            raise ValueError(gp_weights)
        self.nodes = gauss_lobatto_nodes(self.k)
        self.gx, self.gw = gauss_legendre(self.k)
        self.cls = classify_cells(self.mesh, self.balls)
        self.active = np.nonzero(self.cls != OUTSIDE)[0]
        self.rank = np.full(self.mesh.n_cells, -1, dtype=np.int64)
        self.rank[self.active] = np.arange(self.active.size)
        self.n_dofs = self.active.size * self.nd
        self.inside_cells = [int(b) for b in self.active if self.cls[b] == INSIDE]
        self.cut_cells = [int(b) for b in self.active if self.cls[b] == CUT]
        self.faces = active_faces(self.mesh, self.balls, self.cls)
        if gp_kind not in ("face", "volume", "volume_all"):
            raise ValueError(gp_kind)
        self.gp_kind = gp_kind
        self.tau_v = gp_gamma
        self._cell_rules = {}
        self._face_rules = {}
        self._layout = None
        # faces touching each active cell
        self.cell_faces = {int(b): [] for b in self.active}
        for fi, (bm, bp, a, kind, gp) in enumerate(self.faces):
            self.cell_faces[bm].append(fi)
            self.cell_faces[bp].append(fi)
        if gp_kind == "volume":
            patch = self.stable_patches()
            self.faces = [(bm, bp, a, kind, fi in patch) for fi, (bm, bp, a, kind, gp) in enumerate(self.faces)]

    def volume_fraction(self, b):
        """|T cap Omega| / |T|: 1 for inside cells, the sum of the reference
        weights of the volume rule for cut cells."""
        if self.cls[b] == INSIDE:
            return 1.0
        return float(np.sum(self.cell_rule(b)[1]))

    def stable_patches(self):
        """Face indices of the stable-neighbour patches: each cut cell with
        its face neighbour of largest volume fraction (slots 2 axis + side in
        increasing order, a later slot winning only by more than 1e-10)."""
        out = set()
        for b in self.cut_cells:
            ijk = self.mesh.index_to_ijk(b)
            best, best_f, best_fi = None, 0.0, None
            for a in range(self.dim):
                for side in (0, 1):
                    if (side == 0 and ijk[a] == 0) or (side == 1 and ijk[a] == self.mesh.n - 1):
                        continue
                    nb = b + (1 if side else -1) * self.mesh.strides[a]
                    if self.cls[nb] == OUTSIDE:
                        continue
                    fr = self.volume_fraction(nb)
                    if best is None or fr > best_f + 1e-10:
                        lo_c, hi_c = (b, nb) if side else (nb, b)
                        fi = next(f for f in self.cell_faces[b] if self.faces[f][0] == lo_c and self.faces[f][1] == hi_c)
                        best, best_f, best_fi = nb, fr, fi
            if best_fi is not None:
                out.add(best_fi)
        return out

    # ---------------------------------------------------------------- rules
    def cell_rule(self, b):
        """Reference-coordinate volume and interface rules of cut cell b."""
        if b not in self._cell_rules:
            lo, hi = self.mesh.cell_box(b)
            vp, vw, sp, sw, sn = self.saye.cell_rule(lo, hi)
            h = self.h
            d = self.dim
            xi_v = (vp - lo) / h if vp.size else np.zeros((0, d))
            xi_s = (sp - lo) / h if sp.size else np.zeros((0, d))
            self._cell_rules[b] = (
                xi_v,
                vw / h**d if vw.size else np.zeros(0),
                xi_s,
                sw / h ** (d - 1) if sw.size else np.zeros(0),
                sn if sn.size else np.zeros((0, d)),
            )
        return self._cell_rules[b]

    def face_rule(self, fi):
        """In-face reference coordinates (free axes in increasing order) and
        reference weights of face fi; structured faces get the Gauss rule."""
        if fi not in self._face_rules:
            bm, bp, a, kind, gp = self.faces[fi]
            d = self.dim
            if kind == "cut":
                lo, hi = self.mesh.cell_box(bm)
                pts, w = self.saye.face_rule(lo, hi, a, hi[a])
                fr = [x for x in range(d) if x != a]
                xi = (pts[:, fr] - lo[fr]) / self.h if pts.size else np.zeros((0, d - 1))
                self._face_rules[fi] = (xi, w / self.h ** (d - 1) if w.size else np.zeros(0))
            else:
                self._face_rules[fi] = self.full_face_rule()
        return self._face_rules[fi]

    def full_face_rule(self):
        d = self.dim
        m = d - 1
        k = self.k
        xi = np.zeros((k**m, m))
        w = np.ones(k**m)
        for idx in range(k**m):
            rem = idx
            for j in range(m):
                g = rem % k
                rem //= k
                xi[idx, j] = self.gx[g]
                w[idx] *= self.gw[g]
        return xi, w

    def full_cell_rule(self):
        d = self.dim
        k = self.k
        xi = np.zeros((k**d, d))
        w = np.ones(k**d)
        for idx in range(k**d):
            rem = idx
            for j in range(d):
                g = rem % k
                rem //= k
                xi[idx, j] = self.gx[g]
                w[idx] *= self.gw[g]
        return xi, w

    # ---------------------------------------------------------------- basis
    def basis(self, xi, deriv_axis=None, order=1):
        """Values (deriv_axis None) or derivative of order ``order`` along
        ``deriv_axis`` of all k^d basis functions at the points xi: (nq, k^d)."""
        vals = []
        for a in range(self.dim):
            D = lagrange_derivatives(self.nodes, xi[:, a], order if a == deriv_axis else 0)
            vals.append(D[order] if a == deriv_axis else D[0])
        return _tensor_product(vals)

    def grad_basis(self, xi):
        """(nq, k^d, d) reference gradients."""
        return np.stack([self.basis(xi, a, 1) for a in range(self.dim)], axis=2)

    def _cached(self, key, fn):
        # tables of the (shared) tensor-product rules are computed once
        if not hasattr(self, "_tables"):
            self._tables = {}
        if key not in self._tables:
            self._tables[key] = fn()
        return self._tables[key]

    def _face_points(self, xi_f, axis, side_value):
        nq = xi_f.shape[0]
        X = np.zeros((nq, self.dim))
        fr = [x for x in range(self.dim) if x != axis]
        X[:, fr] = xi_f
        X[:, axis] = side_value
        return X

    # ---------------------------------------------------------------- layout
    def layout(self):
        """Offsets of every entity's quadrature points in the kappa vector."""
        if self._layout is None:
            nd = self.nd
            nf = self.k ** (self.dim - 1)
            off = 0
            vol = {}
            for b in self.inside_cells:
                vol[b] = (off, nd)
                off += nd
            seg_cut = off
            for b in self.cut_cells:
                n = self.cell_rule(b)[0].shape[0]
                vol[b] = (off, n)
                off += n
            seg_fstr = off
            face = {}
            for fi, f in enumerate(self.faces):
                if f[3] == "str":
                    face[fi] = (off, nf)
                    off += nf
            seg_fcut = off
            for fi, f in enumerate(self.faces):
                if f[3] == "cut":
                    n = self.face_rule(fi)[0].shape[0]
                    face[fi] = (off, n)
                    off += n
            seg_surf = off
            surf = {}
            for b in self.cut_cells:
                n = self.cell_rule(b)[2].shape[0]
                surf[b] = (off, n)
                off += n
            self._layout = dict(
                vol=vol,
                face=face,
                surf=surf,
                n_qp=off,
                segments=(0, seg_cut, seg_fstr, seg_fcut, seg_surf, off),
            )
        return self._layout

    def qp_physical_points(self):
        """Physical coordinates of every quadrature point in kappa order."""
        L = self.layout()
        P = np.zeros((L["n_qp"], self.dim))
        h = self.h
        for b, (o, n) in L["vol"].items():
            lo, _ = self.mesh.cell_box(b)
            xi = self.full_cell_rule()[0] if self.cls[b] == INSIDE else self.cell_rule(b)[0]
            P[o : o + n] = lo + h * xi
        for fi, (o, n) in L["face"].items():
            bm, bp, a, kind, gp = self.faces[fi]
            lo, _ = self.mesh.cell_box(bm)
            X = self._face_points(self.face_rule(fi)[0], a, 1.0)
            P[o : o + n] = lo + h * X
        for b, (o, n) in L["surf"].items():
            lo, _ = self.mesh.cell_box(b)
            P[o : o + n] = lo + h * self.cell_rule(b)[2]
        return P

    # ---------------------------------------------------------------- apply
    def _cells_of_interest(self, cells):
        if cells is None:
            return set(int(b) for b in self.active)
        return set(int(b) for b in cells)

    def apply(self, u, mask=ALL, kappa=None, cells=None):
        """v = A u.  With ``cells`` (background indices) only the rows of
        those cells are computed; the other rows stay zero."""
        return self._evaluate(u, u, mask, kappa, cells, want_dkappa=False)[0]

    def dkappa(self, w, u, cells=None):
        """dL/dkappa_q = a_q(w, u), the quadrature-point contribution of the
        kappa-weighted terms to w^T A u (ghost penalty carries no kappa).
        With ``cells`` (background indices) only the points of those cells
        and of the faces touching them are computed; the others stay zero."""
        return self._evaluate(w, u, ALL, None, cells, want_dkappa=True)[1]

    def _block(self, vec, b):
        r = self.rank[b]
        return vec[r * self.nd : (r + 1) * self.nd]

    def _evaluate(self, w, u, mask, kappa, cells, want_dkappa):
        targets = self._cells_of_interest(cells)
        v = np.zeros(self.n_dofs)
        need_layout = kappa is not None or want_dkappa
        L = self.layout() if need_layout else None
        dk = np.zeros(L["n_qp"]) if want_dkappa else None
        s = self.h ** (self.dim - 2)

        def kap(o, n):
            if kappa is None:
                return np.ones(n)
            return np.asarray(kappa[o : o + n], dtype=np.float64)

        # volume and interface terms, cell by cell
        for b in sorted(targets):
            ub = self._block(u, b)
            wb = self._block(w, b)
            if self.cls[b] == INSIDE:
                xi, wq = self.full_cell_rule()
            else:
                xi, wq, xs, ws, ns = self.cell_rule(b)
            if mask & VOL and xi.shape[0] > 0:
                if self.cls[b] == INSIDE:
                    G = self._cached(("cellgrad",), lambda: self.grad_basis(xi))
                else:
                    G = self.grad_basis(xi)
                gu = np.einsum("qla,l->qa", G, ub)
                o, n = L["vol"][b] if L else (0, xi.shape[0])
                c = s * wq * kap(o, n)
                if b in targets:
                    self._block(v, b)[:] += np.einsum("qla,qa->l", G, c[:, None] * gu)
                if want_dkappa:
                    gw = np.einsum("qla,l->qa", G, wb)
                    dk[o : o + n] += s * wq * np.sum(gw * gu, axis=1)
            if self.cls[b] == CUT and mask & NITSCHE and xs.shape[0] > 0:
                Phi = self.basis(xs)
                G = self.grad_basis(xs)
                uq = Phi @ ub
                dnu = np.einsum("qla,l,qa->q", G, ub, ns)
                dnphi = np.einsum("qla,qa->ql", G, ns)
                o, n = L["surf"][b] if L else (0, xs.shape[0])
                c = s * ws * kap(o, n)
                if b in targets:
                    self._block(v, b)[:] += (
                        -dnphi.T @ (c * uq) - Phi.T @ (c * dnu) + self.tau * (Phi.T @ (c * uq))
                    )
                if want_dkappa:
                    wq_ = Phi @ wb
                    dnw = np.einsum("qla,l,qa->q", G, wb, ns)
                    dk[o : o + n] += s * ws * (-dnw * uq - wq_ * dnu + self.tau * wq_ * uq)

        # face terms
        for fi, (bm, bp, a, kind, gp) in enumerate(self.faces):
            if bm not in targets and bp not in targets:
                continue
            um, up = self._block(u, bm), self._block(u, bp)
            wm, wp = self._block(w, bm), self._block(w, bp)
            if mask & SIPG and kind != "none":
                xf, wf = self.face_rule(fi)
                if xf.shape[0] > 0:
                    Xm = self._face_points(xf, a, 1.0)
                    Xp = self._face_points(xf, a, 0.0)
                    if kind == "str":
                        Pm, Pp, Dm, Dp = self._cached(
                            ("sipg", a),
                            lambda: (self.basis(Xm), self.basis(Xp), self.basis(Xm, a, 1), self.basis(Xp, a, 1)),
                        )
                    else:
                        Pm, Pp = self.basis(Xm), self.basis(Xp)
                        Dm, Dp = self.basis(Xm, a, 1), self.basis(Xp, a, 1)
                    jump = Pm @ um - Pp @ up
                    avg = 0.5 * (Dm @ um + Dp @ up)
                    o, n = L["face"][fi] if L else (0, xf.shape[0])
                    c = s * wf * kap(o, n)
                    if bm in targets:
                        self._block(v, bm)[:] += (
                            -0.5 * Dm.T @ (c * jump) - Pm.T @ (c * avg) + self.gamma * (Pm.T @ (c * jump))
                        )
                    if bp in targets:
                        self._block(v, bp)[:] += (
                            -0.5 * Dp.T @ (c * jump) + Pp.T @ (c * avg) - self.gamma * (Pp.T @ (c * jump))
                        )
                    if want_dkappa:
                        wjump = Pm @ wm - Pp @ wp
                        wavg = 0.5 * (Dm @ wm + Dp @ wp)
                        dk[o : o + n] += s * wf * (-wavg * jump - wjump * avg + self.gamma * wjump * jump)
            if mask & GP and gp and self.gp_kind != "face":
                self._volume_gp(fi, um, up, v, targets)
            elif mask & GP and gp:
                xf, wf = self.full_face_rule()
                Xm = self._face_points(xf, a, 1.0)
                Xp = self._face_points(xf, a, 0.0)
                for j in self.gp_j:
                    if j == 0:
                        Dm, Dp = self._cached(("gp", a, 0), lambda: (self.basis(Xm), self.basis(Xp)))
                    else:
                        Dm, Dp = self._cached(
                            ("gp", a, j), lambda: (self.basis(Xm, a, j), self.basis(Xp, a, j))
                        )
                    jump = Dm @ um - Dp @ up
                    c = s * self.gp_w[j] * wf
                    if bm in targets:
                        self._block(v, bm)[:] += Dm.T @ (c * jump)
                    if bp in targets:
                        self._block(v, bp)[:] -= Dp.T @ (c * jump)
        return v, dk

    def _volume_gp(self, fi, um, up, v, targets):
        """The patch of face fi (lower cell bm, upper cell bp at +e_axis):
        tau_v h^(d-2) sum over both cells' Gauss points of w J(phi_i) J(u),
        J u = u_bm - u_bp with each polynomial evaluated at the point in its
        own reference coordinates (the shifted points)."""
        bm, bp, a, kind, gp = self.faces[fi]
        xi, wq = self.full_cell_rule()
        shift = np.zeros(self.dim)
        shift[a] = 1.0
        c = self.tau_v * self.h ** (self.dim - 2) * wq
        for pts_m in (xi, xi + shift):  # the Gauss points of bm, then of bp, in bm's coordinates
            Pm = self.basis(pts_m)
            Pp = self.basis(pts_m - shift)
            jump = Pm @ um - Pp @ up
            if bm in targets:
                self._block(v, bm)[:] += Pm.T @ (c * jump)
            if bp in targets:
                self._block(v, bp)[:] -= Pp.T @ (c * jump)

    # ------------------------------------------------------------ utilities
    def dof_values_of(self, fn):
        """Nodal interpolation of a function of physical coordinates."""
        out = np.zeros(self.n_dofs)
        k = self.k
        for b in self.active:
            lo, _ = self.mesh.cell_box(int(b))
            for l in range(self.nd):
                rem = l
                x = np.zeros(self.dim)
                for a in range(self.dim):
                    x[a] = lo[a] + self.h * self.nodes[rem % k]
                    rem //= k
                out[self.rank[b] * self.nd + l] = fn(x)
        return out

    def assemble(self, mask=ALL, kappa=None):
        """Dense matrix by applying the operator to unit vectors (the local
        matrices of Section 3.1 obtained column by column).  Small meshes."""
        A = np.zeros((self.n_dofs, self.n_dofs))
        e = np.zeros(self.n_dofs)
        for j in range(self.n_dofs):
            e[j] = 1.0
            A[:, j] = self.apply(e, mask, kappa)
            e[j] = 0.0
        return A

    def stats(self):
        return dict(
            n_active=int(self.active.size),
            n_inside=len(self.inside_cells),
            n_cut=len(self.cut_cells),
            n_faces=len(self.faces),
            n_dofs=int(self.n_dofs),
        )


def from_workload(wl, **kw):
    return UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, wl.lo, wl.hi, **kw)


class UnfittedCG:
    """The continuous Q_p space (FE_Q) on the same mesh, level set and
    quadrature (Section 2.1, eq. bilinear_cg: Poisson and Nitsche terms; the
    ghost penalty as for DG; no interior-face term).

    DoFs are the Gauss-Lobatto nodes of the active cells on the global node
    lattice ((n p + 1)^d nodes, node (I_0, .., I_{d-1}) at lo + h I / p),
    numbered in lattice order (I_0 fastest).  A continuous function is the
    same polynomial on both sides of every face, so its cell DoFs are its
    node values copied into each cell (u_cell = P u), and the form, being a
    sum of cell, interface and face integrals, is

        A_CG = P^T A_cell P,

    A_cell the cell-DoF operator of UnfittedDG without the SIPG term (which
    vanishes on continuous test and trial functions anyway).
    """

    def __init__(self, *args, **kw):
        self.dg = UnfittedDG(*args, **kw)
        dg = self.dg
        self.dim, self.p, self.k, self.nd, self.h = dg.dim, dg.p, dg.k, dg.nd, dg.h
        L1 = dg.mesh.n * dg.p + 1
        lat = np.zeros((dg.active.size, dg.nd), dtype=np.int64)
        for r, b in enumerate(dg.active):
            ijk = dg.mesh.index_to_ijk(int(b))
            for l in range(dg.nd):
                g, stride, rem = 0, 1, l
                for a in range(dg.dim):
                    g += (ijk[a] * dg.p + rem % dg.k) * stride
                    rem //= dg.k
                    stride *= L1
                lat[r, l] = g
        self.lattice = np.unique(lat)  # active nodes in lattice order
        self.cell_node = np.searchsorted(self.lattice, lat.reshape(-1))
        self.n_dofs = self.lattice.size
        self.L1 = L1

    def gather(self, u):
        """P u: node values into the cells' DoFs."""
        return np.asarray(u, dtype=np.float64)[self.cell_node]

    def scatter(self, v_cell):
        """P^T v: each node sums its cells' values."""
        return np.bincount(self.cell_node, weights=v_cell, minlength=self.n_dofs)

    def apply(self, u, mask=ALL, kappa=None):
        return self.scatter(self.dg.apply(self.gather(u), mask & ~SIPG, kappa))

    def dkappa(self, w, u):
        """dL/dkappa_q of the continuous operator (the SIPG points of the
        kappa layout carry no term: 0)."""
        return self.dg._evaluate(self.gather(w), self.gather(u), ALL & ~SIPG, None, None, want_dkappa=True)[1]

    def node_points(self):
        """Physical coordinates of the nodes."""
        nodes = gauss_lobatto_nodes(self.k)
        X = np.zeros((self.n_dofs, self.dim))
        rem = self.lattice.copy()
        for a in range(self.dim):
            I = rem % self.L1
            rem //= self.L1
            c, i = np.divmod(I, self.p)
            # the last node of the lattice belongs to the last cell's end
            X[:, a] = self.dg.mesh.lo + self.h * (c + nodes[i])
        return X

    def dof_values_of(self, fn):
        return np.array([fn(x) for x in self.node_points()])
