"""Seeded synthetic inputs shared by the oracle-side tests and the product-side
tests and benchmarks.

This module holds no arithmetic of the method itself: it only draws the
geometry parameters (ball centres and radii), the DoF vectors and the
coefficient samples that both implementations receive as inputs.  Every draw
goes through ``numpy.random.default_rng(seed)`` in a fixed order:
geometry first, then the primary vector (u or u*), then the secondary vectors
(b, w, delta-kappa).

Workloads (all on the box [-1, 1]^d, uniform background mesh of n^d cells):

* ``disk2d``   -- 2D, degree 2, 16^2 cells, disk of radius 0.7 whose centre is
  offset by a draw uniform in [-0.05, 0.05]^2.
* ``ball3d``   -- 3D, degree 3, 64^3 cells, ball of radius 0.8 whose centre
  offset is drawn uniform in [-0.05, 0.05]^3 and redrawn until its length is
  at most 0.05.
* ``sweep3d``  -- 3D, degree p = 1..7 on the ball geometry above, background
  resolution chosen so that the active DoF count is about 2e7.
* ``kappa3d``  -- 3D, degree 4, 48^3 cells, ball geometry above, variable
  coefficient kappa(x) = 1 + 0.5 sin(pi x) sin(pi y) sin(pi z).
* ``balls3d``  -- 3D, degree 3, 128^3 cells, union of 20 balls with centres
  uniform in [-0.7, 0.7]^3 and radii uniform in [0.1, 0.3].
* ``plane3d``  -- the plane benchmark (Section 5.2): 3D, degree 1 or 3, n^3
  cells, domain below a plane z ~ const whose normal is tilted by (1e-3,
  2e-3) and whose position lies in layer L of the cells (a seeded offset
  within the middle third of the layer): layers below are inside, layer L
  is cut, so the ratio of cut to physical cells is 1 / (L + 1); L = n puts
  the plane above the box (no cut cell).

The paper measures on spheres and random sphere unions of its own (Section 6);
these seeded geometries stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Background resolution per degree for the degree sweep: about 2e7 active DoF
# on the radius-0.8 ball.
SWEEP_N = {1: 209, 2: 139, 3: 104, 4: 83, 5: 69, 6: 59, 7: 51}


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    n: int
    degree: int
    centers: np.ndarray  # (m, dim) float64
    radii: np.ndarray  # (m,) float64
    seed: int
    lo: float = -1.0
    hi: float = 1.0
    plane: tuple | None = None  # (normal, offset): level set n . x - offset instead of balls

    @property
    def h(self) -> float:
        return (self.hi - self.lo) / self.n


def _ball_offset(rng: np.random.Generator, dim: int, bound: float = 0.05) -> np.ndarray:
    while True:
        off = rng.uniform(-bound, bound, size=dim)
        if float(np.sqrt(np.sum(off * off))) <= bound:
            return off


def make_rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def disk2d(seed: int = 0, n: int = 16, degree: int = 2, radius: float = 0.7):
    rng = make_rng(seed)
    off = rng.uniform(-0.05, 0.05, size=2)
    wl = Workload("disk2d", 2, n, degree, off.reshape(1, 2).copy(), np.array([radius]), seed)
    return wl, rng


def ball3d(seed: int = 0, n: int = 64, degree: int = 3, radius: float = 0.8, name: str = "ball3d"):
    rng = make_rng(seed)
    off = _ball_offset(rng, 3)
    wl = Workload(name, 3, n, degree, off.reshape(1, 3).copy(), np.array([radius]), seed)
    return wl, rng


def sweep3d(degree: int, seed: int = 0, n: int | None = None):
    return ball3d(seed=seed, n=n if n is not None else SWEEP_N[degree], degree=degree, name="sweep3d")


def kappa3d(seed: int = 0, n: int = 48, degree: int = 4):
    return ball3d(seed=seed, n=n, degree=degree, name="kappa3d")


def balls3d(seed: int = 0, n: int = 128, degree: int = 3, n_balls: int = 20):
    rng = make_rng(seed)
    centers = rng.uniform(-0.7, 0.7, size=(n_balls, 3))
    radii = rng.uniform(0.1, 0.3, size=n_balls)
    wl = Workload("balls3d", 3, n, degree, centers, radii, seed)
    return wl, rng


def custom(dim: int, n: int, degree: int, centers, radii, seed: int = 0, name: str = "custom"):
    rng = make_rng(seed)
    c = np.asarray(centers, dtype=np.float64).reshape(-1, dim)
    r = np.asarray(radii, dtype=np.float64).reshape(-1)
    return Workload(name, dim, n, degree, c, r, seed), rng


def plane(dim: int, n: int, degree: int, normal, offset, seed: int = 0, name: str = "plane"):
    rng = make_rng(seed)
    nv = np.asarray(normal, dtype=np.float64).reshape(-1)
    return Workload(name, dim, n, degree, np.zeros((0, dim)), np.zeros(0), seed,
                    plane=(nv, float(offset))), rng


PLANE_TILT = (1e-3, 2e-3)


def plane3d(layer: int, seed: int = 0, n: int = 128, degree: int = 1):
    """Plane benchmark: cut-cell ratio 1 / (layer + 1) (0 for layer >= n)."""
    rng = make_rng(seed)
    h = 2.0 / n
    jitter = rng.uniform(-h / 6, h / 6)
    if layer >= n:
        offset = 1.5
    else:
        offset = -1.0 + (layer + 0.5) * h + jitter
    nv = np.array([PLANE_TILT[0], PLANE_TILT[1], 1.0])
    wl = Workload("plane3d", 3, n, degree, np.zeros((0, 3)), np.zeros(0), seed, plane=(nv, offset))
    return wl, rng


def uniform_vector(rng: np.random.Generator, n: int) -> np.ndarray:
    """Entries uniform in [-1, 1], float64."""
    return rng.uniform(-1.0, 1.0, size=n)


def kappa_field(points: np.ndarray) -> np.ndarray:
    """Coefficient samples 1 + 0.5 sin(pi x) sin(pi y) sin(pi z) at physical
    points (rows of ``points``; 2D uses the first two factors)."""
    pts = np.asarray(points, dtype=np.float64)
    val = np.ones(pts.shape[0])
    s = np.ones(pts.shape[0])
    for a in range(pts.shape[1]):
        s = s * np.sin(math.pi * pts[:, a])
    return val + 0.5 * s


BY_NAME = {
    "disk2d": disk2d,
    "ball3d": ball3d,
    "kappa3d": kappa3d,
    "balls3d": balls3d,
}
