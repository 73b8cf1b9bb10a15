"""Dimension-reduction quadrature on cut cells, cut faces and the interface.

Test infrastructure only (see the package docstring).

The paper generates its unstructured quadrature with the dimension-reduction
method of Saye (2015), cited in Sections 1 and 2.3, and notes that cut-cell
refinement multiplies the point count by 2^(d n_ref) (Section 5.1).  The paper
prints no steps of its own, so this module follows the published method, read
as follows for level sets that are unions of balls:

TOP problem on a box U (integrate over {phi < 0} inside U):
  1. If some ball contains U, use the tensor Gauss rule on U.  Balls that stay
     away from U (distance >= R) are dropped; if none is left U is empty.
  2. Height direction: among the free axes along which every remaining ball
     function is strictly monotone on U (the centre coordinate lies outside
     [lo_k, hi_k]), take the one with the largest sum of |d psi_i / d x_k| at
     the box centre; ties go to the lowest axis.
  3. If there is none, bisect U along every free axis and recurse (children
     in binary order, first free axis = lowest bit), at most ``max_depth``
     times; at the depth limit use the tensor rule on U and keep the points
     with phi < 0 (no interface points there).
  4. Otherwise build a quadrature of the whole lower face U' (U without axis
     k), split at the zero sets of every ball function restricted to
     x_k = lo_k and x_k = hi_k (the SPLIT problem below).
  5. For each base point, the line along k is split at the roots of the ball
     functions (solved in closed form); a Gauss rule with q points is placed on
     each piece whose midpoint has phi < 0.  Each root where the root's ball is
     the active minimum is an interface point with weight
     w' |grad psi| / |d psi / d x_k| and unit normal grad psi / |grad psi|.
SPLIT problem on a box (integrate over the whole box):
  functions with one sign on the box are dropped; with none left, or in one
  dimension, Gauss rules go on the pieces between the roots; otherwise steps
  2-5 apply with every piece kept.

Every rule uses q Gauss-Legendre points per one-dimensional piece.

A plane level set psi = n . x - c (one function, unit n) takes the same
steps: its bounds on a box are the smallest and largest values at the
corners, it is strictly monotone along every axis with n_k != 0, the height
criterion |d psi / d x_k| / |grad psi| is |n_k|, the root along a line is
(c - sum over the other axes of n_a x_a) / n_k, and an interface point has
weight w' / |n_k| and normal n.
"""
from __future__ import annotations

import math

import numpy as np

from .basis import gauss_legendre
from .geometry import Plane


class SayeQuadrature:
    def __init__(self, balls, dim: int, q: int, max_depth: int = 4):
        self.balls = balls
        self.plane = isinstance(balls, Plane)
        self.dim = dim
        self.q = q
        self.max_depth = max_depth
        self.gx, self.gw = gauss_legendre(q)
        self.n_fallback = 0

    # -- function helpers; a function is (ball index, vals) where vals holds
    # -- the coordinates of every axis that is not free in the current box.
    def _coord(self, f, x, free, a):
        return x[a] if a in free else f[1][a]

    def _bounds(self, f, lo, hi, free):
        i, vals = f
        if self.plane:
            nv = self.balls.n
            mn = 0.0
            mx = 0.0
            for a in range(self.dim):
                if a in free:
                    mn += nv[a] * lo[a] if nv[a] > 0 else nv[a] * hi[a]
                    mx += nv[a] * hi[a] if nv[a] > 0 else nv[a] * lo[a]
                else:
                    mn += nv[a] * vals[a]
                    mx += nv[a] * vals[a]
            return mn - self.balls.c0, mx - self.balls.c0
        c = self.balls.c[i]
        near2 = 0.0
        far2 = 0.0
        for a in range(self.dim):
            if a in free:
                nz = min(max(c[a], lo[a]), hi[a]) - c[a]
                fz = max(abs(lo[a] - c[a]), abs(hi[a] - c[a]))
            else:
                nz = vals[a] - c[a]
                fz = abs(vals[a] - c[a])
            near2 += nz * nz
            far2 += fz * fz
        r = self.balls.r[i]
        return math.sqrt(near2) - r, math.sqrt(far2) - r

    def _psi(self, f, x, free):
        i, vals = f
        if self.plane:
            nv = self.balls.n
            s = 0.0
            for a in range(self.dim):
                s += nv[a] * self._coord(f, x, free, a)
            return s - self.balls.c0
        c = self.balls.c[i]
        s = 0.0
        for a in range(self.dim):
            z = self._coord(f, x, free, a) - c[a]
            s += z * z
        return math.sqrt(s) - self.balls.r[i]

    def _monotone(self, f, k, lo, hi):
        if self.plane:
            return self.balls.n[k] != 0.0
        ck = self.balls.c[f[0]][k]
        return ck < lo[k] or ck > hi[k]

    def _height(self, funcs, lo, hi, free):
        best, bestval = None, -1.0
        for k in sorted(free):
            if not all(self._monotone(f, k, lo, hi) for f in funcs):
                continue
            val = 0.0
            for f in funcs:
                i, vals = f
                if self.plane:
                    val += abs(self.balls.n[k])
                    continue
                c = self.balls.c[i]
                s = 0.0
                for a in range(self.dim):
                    xa = 0.5 * (lo[a] + hi[a]) if a in free else vals[a]
                    s += (xa - c[a]) ** 2
                r = math.sqrt(s)
                if r > 0.0:
                    val += abs((0.5 * (lo[k] + hi[k]) - c[k]) / r)
            if val > bestval:
                best, bestval = k, val
        return best

    def _roots(self, funcs, x, free, k, a, b):
        """Roots in (a, b) of the functions along axis k through x, sorted."""
        out = []
        for fi, f in enumerate(funcs):
            i, vals = f
            if self.plane:
                nv = self.balls.n
                if nv[k] == 0.0:
                    continue
                s = 0.0
                for ax in range(self.dim):
                    if ax != k:
                        s += nv[ax] * self._coord(f, x, free, ax)
                t = (self.balls.c0 - s) / nv[k]
                if a < t < b:
                    out.append((t, fi))
                continue
            c = self.balls.c[i]
            s = 0.0
            for ax in range(self.dim):
                if ax == k:
                    continue
                z = self._coord(f, x, free, ax) - c[ax]
                s += z * z
            D = self.balls.r[i] ** 2 - s
            if D < 0.0:
                continue
            sq = math.sqrt(D)
            for t in (c[k] - sq, c[k] + sq):
                if a < t < b:
                    out.append((t, fi))
        out.sort(key=lambda e: e[0])
        return out

    def _tensor(self, lo, hi, free, base):
        fr = sorted(free)
        m = len(fr)
        q = self.q
        pts, wts = [], []
        for idx in range(q**m):
            x = base.copy()
            w = 1.0
            rem = idx
            for a in fr:
                g = rem % q
                rem //= q
                L = hi[a] - lo[a]
                x[a] = lo[a] + L * self.gx[g]
                w *= L * self.gw[g]
            pts.append(x)
            wts.append(w)
        return pts, wts

    def _children(self, lo, hi, free):
        fr = sorted(free)
        for cidx in range(2 ** len(fr)):
            clo, chi = lo.copy(), hi.copy()
            for j, a in enumerate(fr):
                mid = 0.5 * (lo[a] + hi[a])
                if (cidx >> j) & 1:
                    clo[a] = mid
                else:
                    chi[a] = mid
            yield clo, chi

    def _pieces(self, a, b, roots):
        edges = [a] + [t for t, _ in roots] + [b]
        for e0, e1 in zip(edges[:-1], edges[1:]):
            if e1 > e0:
                yield e0, e1

    # -- SPLIT: whole box, cut at the zero sets of funcs --
    def _split(self, funcs, lo, hi, free, base, depth):
        keep = []
        for f in funcs:
            mn, mx = self._bounds(f, lo, hi, free)
            if mn < 0.0 < mx:
                keep.append(f)
        if not keep:
            return self._tensor(lo, hi, free, base)
        fr = sorted(free)
        if len(fr) == 1:
            k = fr[0]
            x = base.copy()
            pts, wts = [], []
            roots = self._roots(keep, x, free, k, lo[k], hi[k])
            for e0, e1 in self._pieces(lo[k], hi[k], roots):
                L = e1 - e0
                for g in range(self.q):
                    y = x.copy()
                    y[k] = e0 + L * self.gx[g]
                    pts.append(y)
                    wts.append(L * self.gw[g])
            return pts, wts
        k = self._height(keep, lo, hi, free)
        if k is None:
            if depth < self.max_depth:
                pts, wts = [], []
                for clo, chi in self._children(lo, hi, free):
                    p2, w2 = self._split(keep, clo, chi, free, base, depth + 1)
                    pts += p2
                    wts += w2
                return pts, wts
            self.n_fallback += 1
            return self._tensor(lo, hi, free, base)
        sub = [a for a in fr if a != k]
        funcs2 = []
        for i, vals in keep:
            vlo = vals.copy()
            vlo[k] = lo[k]
            vhi = vals.copy()
            vhi[k] = hi[k]
            funcs2.append((i, vlo))
            funcs2.append((i, vhi))
        bpts, bwts = self._split(funcs2, lo, hi, set(sub), base, 0)
        pts, wts = [], []
        for x, w in zip(bpts, bwts):
            roots = self._roots(keep, x, free, k, lo[k], hi[k])
            for e0, e1 in self._pieces(lo[k], hi[k], roots):
                L = e1 - e0
                for g in range(self.q):
                    y = x.copy()
                    y[k] = e0 + L * self.gx[g]
                    pts.append(y)
                    wts.append(w * (L * self.gw[g]))
        return pts, wts

    # -- TOP: {phi < 0} inside the box --
    def _top(self, funcs, lo, hi, free, base, depth, want_surface):
        rel = []
        for f in funcs:
            mn, mx = self._bounds(f, lo, hi, free)
            if mx < 0.0:
                p, w = self._tensor(lo, hi, free, base)
                return p, w, [], [], []
            if mn < 0.0:
                rel.append(f)
        if not rel:
            return [], [], [], [], []
        fr = sorted(free)
        vp, vw, sp, sw, sn = [], [], [], [], []
        if len(fr) == 1:
            k = fr[0]
            self._line(rel, base.copy(), 1.0, free, k, lo[k], hi[k], want_surface, vp, vw, sp, sw, sn)
            return vp, vw, sp, sw, sn
        k = self._height(rel, lo, hi, free)
        if k is None:
            if depth < self.max_depth:
                for clo, chi in self._children(lo, hi, free):
                    r = self._top(rel, clo, chi, free, base, depth + 1, want_surface)
                    vp += r[0]
                    vw += r[1]
                    sp += r[2]
                    sw += r[3]
                    sn += r[4]
                return vp, vw, sp, sw, sn
            self.n_fallback += 1
            p, w = self._tensor(lo, hi, free, base)
            for x, ww in zip(p, w):
                if min(self._psi(f, x, free) for f in rel) < 0.0:
                    vp.append(x)
                    vw.append(ww)
            return vp, vw, sp, sw, sn
        sub = [a for a in fr if a != k]
        funcs2 = []
        for i, vals in rel:
            vlo = vals.copy()
            vlo[k] = lo[k]
            vhi = vals.copy()
            vhi[k] = hi[k]
            funcs2.append((i, vlo))
            funcs2.append((i, vhi))
        bpts, bwts = self._split(funcs2, lo, hi, set(sub), base, 0)
        for x, w in zip(bpts, bwts):
            self._line(rel, x, w, free, k, lo[k], hi[k], want_surface, vp, vw, sp, sw, sn)
        return vp, vw, sp, sw, sn

    def _line(self, rel, x, w, free, k, a, b, want_surface, vp, vw, sp, sw, sn):
        roots = self._roots(rel, x, free, k, a, b)
        for e0, e1 in self._pieces(a, b, roots):
            y = x.copy()
            y[k] = 0.5 * (e0 + e1)
            if min(self._psi(f, y, free) for f in rel) < 0.0:
                L = e1 - e0
                for g in range(self.q):
                    y = x.copy()
                    y[k] = e0 + L * self.gx[g]
                    vp.append(y)
                    vw.append(w * (L * self.gw[g]))
        if not want_surface:
            return
        for t, fi in roots:
            y = x.copy()
            y[k] = t
            active = True
            for gi, g in enumerate(rel):
                if gi != fi and self._psi(g, y, free) < 0.0:
                    active = False
                    break
            if not active:
                continue
            if self.plane:
                sp.append(y)
                sw.append(w / abs(self.balls.n[k]))
                sn.append(self.balls.n.copy())
                continue
            i = rel[fi][0]
            c = self.balls.c[i]
            d = np.array([self._coord(rel[fi], y, free, ax) - c[ax] for ax in range(self.dim)])
            r = math.sqrt(float(np.dot(d, d)))
            sp.append(y)
            sw.append(w * (r / abs(t - c[k])))
            sn.append(d / r)

    # -- public entry points --
    def cell_rule(self, lo, hi):
        """Volume and interface rule of the cell box [lo, hi] in physical
        coordinates: (vol_pts, vol_w, surf_pts, surf_w, surf_normals)."""
        lo = np.asarray(lo, dtype=np.float64)
        hi = np.asarray(hi, dtype=np.float64)
        funcs = [(i, lo.copy()) for i in range(self.balls.m)]
        r = self._top(funcs, lo, hi, set(range(self.dim)), lo.copy(), 0, True)
        return tuple(np.array(v, dtype=np.float64) for v in r)

    def face_rule(self, lo, hi, axis: int, value: float):
        """Rule on {phi < 0} of the face x_axis = value of the box [lo, hi]."""
        lo = np.asarray(lo, dtype=np.float64).copy()
        hi = np.asarray(hi, dtype=np.float64).copy()
        base = lo.copy()
        base[axis] = value
        lo[axis] = value
        hi[axis] = value
        free = set(range(self.dim)) - {axis}
        funcs = [(i, base.copy()) for i in range(self.balls.m)]
        r = self._top(funcs, lo, hi, free, base, 0, False)
        return np.array(r[0], dtype=np.float64), np.array(r[1], dtype=np.float64)
