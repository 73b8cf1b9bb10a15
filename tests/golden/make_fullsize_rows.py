"""Write the oracle's rows of sampled cells at the full workload sizes.

Test infrastructure: calls only the oracle (``oracle/``) and the seeded input
generators (``ufem_inputs``); nothing here comes from the HIP library.  The
GPU parity tests regenerate the same seeded vectors, run the library on the
whole mesh in the benchmark's launch configuration and compare the rows of
the sampled cells with the values stored here.

Usage:  python tests/golden/make_fullsize_rows.py [name ...]
        (names: ball3d, balls3d, kappa3d, sweep1 ... sweep7, plane_p<p>_l<layer>;
        default all)

Per workload the file fullsize_<name>.npz holds
  cells      sampled active cells (background indices): random inside and cut
             cells, and where the oracle's full layout is computed, the cut
             cell with the largest volume rule
  n_dofs     active DoF count of the oracle
  rows64     v = A u on those cells' rows (float64 u)
  rows32     v = A u32 (u rounded to float32, evaluated in float64)
  rows_adj   A^T w = A w on those rows (kappa of the workload)
  dk_idx, dk_val   dL/dkappa at every quadrature point of the sampled cells
             and of the faces touching them (ball and kappa workloads)
Draw order as everywhere: geometry, u, then w.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import ufem_inputs as ui  # noqa: E402
from oracle.geometry import INSIDE  # noqa: E402
from oracle.operator import ALL, UnfittedDG  # noqa: E402


def workload(name):
    if name == "ball3d":
        return ui.ball3d(0)
    if name == "balls3d":
        return ui.balls3d(0)
    if name == "kappa3d":
        return ui.kappa3d(0)
    if name.startswith("sweep"):
        return ui.sweep3d(int(name[5:]), 0)
    if name.startswith("plane_p"):
        p, layer = name[7:].split("_l")
        return ui.plane3d(int(layer), 0, n=128, degree=int(p))
    raise ValueError(name)


def make(name, n_inside=4, n_cut=8):
    t0 = time.time()
    wl, rng = workload(name)
    ora = UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, wl.lo, wl.hi, plane=wl.plane)
    print(f"[{name}] oracle built in {time.time() - t0:.0f} s, {ora.n_dofs} DoF", flush=True)
    u = ui.uniform_vector(rng, ora.n_dofs)
    w = ui.uniform_vector(rng, ora.n_dofs)
    pick = np.random.default_rng(7)
    cells = [int(b) for b in pick.choice(ora.inside_cells, min(n_inside, len(ora.inside_cells)), replace=False)]
    cells += [int(b) for b in pick.choice(ora.cut_cells, n_cut, replace=False)]
    with_layout = name in ("ball3d", "balls3d", "kappa3d")
    kap = None
    if with_layout:
        L = ora.layout()
        big = max(ora.cut_cells, key=lambda b: L["vol"][b][1])
        if big not in cells:
            cells.append(int(big))
        if name == "kappa3d":
            kap = ui.kappa_field(ora.qp_physical_points())
    out = {"cells": np.array(cells, dtype=np.int64), "n_dofs": np.int64(ora.n_dofs),
           "degree": np.int64(wl.degree), "n": np.int64(wl.n)}

    def rows(v):
        return np.stack([v[ora.rank[b] * ora.nd:(ora.rank[b] + 1) * ora.nd] for b in cells])

    out["rows64"] = rows(ora.apply(u, ALL, kap, cells=cells))
    u32 = u.astype(np.float32).astype(np.float64)
    out["rows32"] = rows(ora.apply(u32, ALL, kap, cells=cells))
    out["rows_adj"] = rows(ora.apply(w, ALL, kap, cells=cells))
    if name in ("ball3d", "kappa3d"):
        dk = ora.dkappa(w, u, cells=cells)
        idx = []
        for b in cells:
            o, m = L["vol"][b]
            idx.extend(range(o, o + m))
            if ora.cls[b] != INSIDE and b in L["surf"]:
                o, m = L["surf"][b]
                idx.extend(range(o, o + m))
            for fi in ora.cell_faces[b]:
                if fi in L["face"]:
                    o, m = L["face"][fi]
                    idx.extend(range(o, o + m))
        idx = np.unique(np.array(idx, dtype=np.int64))
        out["dk_idx"] = idx
        out["dk_val"] = dk[idx]
    path = os.path.join(HERE, f"fullsize_{name}.npz")
    np.savez_compressed(path, **out)
    print(f"[{name}] wrote {path} ({len(cells)} cells) in {time.time() - t0:.0f} s", flush=True)


def main(argv):
    names = argv or (["ball3d", "kappa3d", "balls3d"] + [f"sweep{p}" for p in range(1, 8)]
                     + ["plane_p1_l0", "plane_p1_l9", "plane_p3_l0", "plane_p3_l1"])
    for nm in names:
        make(nm)


if __name__ == "__main__":
    main(sys.argv[1:])
