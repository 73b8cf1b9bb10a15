"""Level set, cell and face classification on the Cartesian background mesh.

Test infrastructure only (see the package docstring).

Level set (Section 6.1): a ball is phi(x) = |x - c| - R; a union of balls is
the minimum of the ball level sets.  The plane benchmark of Section 5.2 uses a
plane, phi(x) = n . x - c with a unit normal n.  The physical domain is
{phi < 0}.

Cell classes (Section 2.3 and the cell categories of Section 3.4):
  inside  -- some single ball contains the closed cell box,
  outside -- every ball stays at distance >= R from the closed box,
  cut     -- otherwise;
for a plane: inside if phi < 0 at every corner of the closed box, outside if
phi >= 0 at every corner, cut otherwise (the same rule: max phi < 0 inside,
min phi >= 0 outside).
Active cells are inside + cut; only they carry DoFs (outside cells get
weight 0 in the paper's load balancing, Section 3.5).

Faces: every interior face between two active cells, ordered by the
background index of the lower cell and then by axis.  A face is
  'str'  (structured SIPG quadrature) if some ball contains it,
  'none' (no SIPG term) if it lies outside every open ball,
  'cut'  otherwise (SIPG with dimension-reduction quadrature).
The ghost penalty acts on the full face whenever one of its cells is cut.
"""
from __future__ import annotations

import math

import numpy as np

INSIDE, CUT, OUTSIDE = 0, 1, 2


class Balls:
    """Union of balls min_i(|x - c_i| - R_i)."""

    def __init__(self, centers, radii):
        self.c = np.asarray(centers, dtype=np.float64)
        self.r = np.asarray(radii, dtype=np.float64).reshape(-1)
        if self.c.ndim != 2 or self.c.shape[0] != self.r.size:
            raise ValueError("centers must be (m, d) and radii (m,)")

    @property
    def m(self) -> int:
        return self.r.size

    def psi(self, i: int, x: np.ndarray) -> float:
        d = x - self.c[i]
        return float(np.sqrt(np.dot(d, d))) - self.r[i]

    def phi(self, x: np.ndarray) -> float:
        return min(self.psi(i, x) for i in range(self.m))

    def phi_many(self, X: np.ndarray) -> np.ndarray:
        X = np.atleast_2d(X)
        best = np.full(X.shape[0], np.inf)
        for i in range(self.m):
            d = X - self.c[i]
            best = np.minimum(best, np.sqrt(np.sum(d * d, axis=1)) - self.r[i])
        return best

    def box_dist(self, i: int, lo: np.ndarray, hi: np.ndarray):
        """Nearest and farthest distance from centre i to the box [lo, hi]."""
        c = self.c[i]
        near = np.clip(c, lo, hi) - c
        far = np.maximum(np.abs(lo - c), np.abs(hi - c))
        return float(np.sqrt(np.dot(near, near))), float(np.sqrt(np.dot(far, far)))


class Plane:
    """Half space below a plane: phi(x) = n . x - c, n of unit length (the
    given normal and offset are scaled by 1 / |normal|)."""

    def __init__(self, normal, offset):
        nv = np.asarray(normal, dtype=np.float64).reshape(-1)
        s = 0.0
        for a in range(nv.size):
            s += float(nv[a]) * float(nv[a])
        L = math.sqrt(s)
        if not L > 0.0:
            raise ValueError("plane normal must be nonzero")
        self.n = nv / L
        self.c0 = float(offset) / L

    @property
    def m(self) -> int:
        return 1

    def psi(self, i: int, x: np.ndarray) -> float:
        s = 0.0
        for a in range(self.n.size):
            s += float(self.n[a]) * float(x[a])
        return s - self.c0

    def phi(self, x: np.ndarray) -> float:
        return self.psi(0, x)

    def phi_many(self, X: np.ndarray) -> np.ndarray:
        X = np.atleast_2d(X)
        return X @ self.n - self.c0

    def box_range(self, lo, hi):
        """Smallest and largest phi over the box [lo, hi]."""
        lo = np.asarray(lo, dtype=np.float64)
        hi = np.asarray(hi, dtype=np.float64)
        mn = float(np.sum(np.where(self.n > 0, self.n * lo, self.n * hi))) - self.c0
        mx = float(np.sum(np.where(self.n > 0, self.n * hi, self.n * lo))) - self.c0
        return mn, mx


def box_class(balls, lo, hi) -> int:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    if isinstance(balls, Plane):
        mn, mx = balls.box_range(lo, hi)
        return INSIDE if mx < 0.0 else (CUT if mn < 0.0 else OUTSIDE)
    any_touch = False
    for i in range(balls.m):
        dmin, dmax = balls.box_dist(i, lo, hi)
        if dmax < balls.r[i]:
            return INSIDE
        if dmin < balls.r[i]:
            any_touch = True
    return CUT if any_touch else OUTSIDE


class Mesh:
    """Uniform background mesh of n^dim cells on [lo, hi]^dim."""

    def __init__(self, dim: int, n: int, lo: float = -1.0, hi: float = 1.0):
        self.dim = dim
        self.n = n
        self.lo = float(lo)
        self.hi = float(hi)
        self.h = (self.hi - self.lo) / n
        self.strides = [n**a for a in range(dim)]
        self.n_cells = n**dim

    def index_to_ijk(self, b: int):
        out = []
        for _ in range(self.dim):
            out.append(b % self.n)
            b //= self.n
        return out

    def cell_box(self, b: int):
        ijk = np.array(self.index_to_ijk(b), dtype=np.float64)
        lo = self.lo + ijk * self.h
        return lo, lo + self.h


def classify_cells(mesh: Mesh, balls) -> np.ndarray:
    """Class of every background cell (vectorised over cells, loop over balls)."""
    idx = np.indices((mesh.n,) * mesh.dim).reshape(mesh.dim, -1)[::-1].T  # x fastest
    lo = mesh.lo + idx * mesh.h
    hi = lo + mesh.h
    if isinstance(balls, Plane):
        nv = balls.n
        mn = np.sum(np.where(nv > 0, nv * lo, nv * hi), axis=1) - balls.c0
        mx = np.sum(np.where(nv > 0, nv * hi, nv * lo), axis=1) - balls.c0
        cls = np.full(mesh.n_cells, OUTSIDE, dtype=np.int8)
        cls[mn < 0.0] = CUT
        cls[mx < 0.0] = INSIDE
        return cls
    inside = np.zeros(mesh.n_cells, dtype=bool)
    touch = np.zeros(mesh.n_cells, dtype=bool)
    for i in range(balls.m):
        c = balls.c[i]
        near = np.clip(c, lo, hi) - c
        far = np.maximum(np.abs(lo - c), np.abs(hi - c))
        dmin = np.sqrt(np.sum(near * near, axis=1))
        dmax = np.sqrt(np.sum(far * far, axis=1))
        inside |= dmax < balls.r[i]
        touch |= dmin < balls.r[i]
    cls = np.full(mesh.n_cells, OUTSIDE, dtype=np.int8)
    cls[touch] = CUT
    cls[inside] = INSIDE
    return cls


def active_faces(mesh: Mesh, balls, cls: np.ndarray):
    """Interior faces between active cells, in canonical order.

    Returns a list of tuples (b_minus, b_plus, axis, kind, gp) where kind is
    'str', 'cut' or 'none' and gp tells whether the ghost penalty acts on it.
    """
    faces = []
    active = np.nonzero(cls != OUTSIDE)[0]
    for b in active:
        ijk = mesh.index_to_ijk(int(b))
        for a in range(mesh.dim):
            if ijk[a] + 1 >= mesh.n:
                continue
            bp = int(b) + mesh.strides[a]
            if cls[bp] == OUTSIDE:
                continue
            lo, hi = mesh.cell_box(int(b))
            flo = lo.copy()
            flo[a] = hi[a]
            fhi = hi.copy()
            fc = box_class(balls, flo, fhi)
            kind = {INSIDE: "str", CUT: "cut", OUTSIDE: "none"}[fc]
            gp = bool(cls[b] == CUT or cls[bp] == CUT)
            faces.append((int(b), bp, a, kind, gp))
    return faces
