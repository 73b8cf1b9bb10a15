#!/usr/bin/env python
"""Benchmark of the matrix-free unfitted DG operator on one MI355X.

Workload (default): 3D SIPG DG, degree 3, 64^3 background cells on [-1, 1]^3,
ball of radius 0.8 with a seeded centre offset (|offset| <= 0.05), Nitsche
terms and face ghost penalty; 4^3 Gauss points on inside cells and
dimension-reduction quadrature with 4 points per 1D piece on cut cells;
u uniform in [-1, 1].  Synthetic, seeded.

One timed step = FP64 apply v = A u, FP32 apply, FP64 adjoint pass (A^T w and
dL/dkappa at every quadrature point), all on vectors resident in HBM.  Several
(u, v) pairs totalling more than the 256 MB last-level cache are rotated so
that every apply streams its vectors from HBM.

`value` is the FP64 operator throughput in active DoF/s (the paper's
throughput metric, Section 5.1: DoFs / time of one operator evaluation); the
FP32 and adjoint throughputs are reported beside it.  Every kernel of a step is
bracketed by HIP events on the stream the library launches on.

Beside the timed steps (not timed): the error of the FP64 and FP32 applies and
of the adjoint pass against the FP64 oracle on sampled rows, the oracle's own
throughput on one core and on every core of the process (at most 16), and
the solve of A u = b to 1e-10 by FP64 CG and by FP32-inner defect correction.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "operator DoF/s (3D DG k=3, FP64 vs FP32) + adjoint DoF/s; % of HBM roofline"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64, published
KERNEL_SOURCES = ["paper_2404_07911_amd/csrc/kernels_impl.hpp", "paper_2404_07911_amd/csrc/device.hpp"]


def progress(msg):
    """a line on stderr per stage, so that a long run shows it is alive"""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# kernel stages of one apply (ufem_apply_part masks): the Kronecker kernel over
# inside cells and the structured faces of cut cells (one launch), the
# volume / interface lines, the cut-face lines
STAGES = {3: "structured", 4: "cut_lines", 8: "cut_face_lines"}
STAGE_KERNELS = {
    "structured": "inside_kron_kernel (inside cells; structured faces and ghost penalty of cut cells)",
    "cut_lines": "cut_batch_kernel (volume and interface lines)",
    "cut_face_lines": "cut_face_kernel (cut-face lines)",
}
STAGE_KERNELS_MIXED = dict(STAGE_KERNELS, cut_lines="cut_matrix_kernel (element matrices of the cut cells)")


def model(info, dim, p, s, kappa=False, mixed=False):
    """Algorithmic bytes per kernel stage and model FLOPs of one apply.

    Bytes (s = bytes per value) count what a stage must move at the least:
    the rows of u it reads and of v it writes for its own cells (structured:
    read u, write v of inside and cut cells; the two line stages add to v, so
    read u, read and write v of cut cells), and the quadrature data of the cut cells
    (volume point: dim coordinates and a weight; interface point: dim
    coordinates, a weight and dim normal components; cut-face point: dim - 1
    in-face coordinates and a weight), plus one kappa value per quadrature
    point when a coefficient field is set.  Index tables are not counted.
    FLOPs: the paper's operation counts (Section 5.1) for 3D: 24 k^4 per
    structured cell, 56 k^3 per structured face (both sides, evaluation and
    integration), 4 (2k^3 + 3k^2 + 4k) per unstructured cell or interface
    point, 8 (k^3 + n_q (3k^2 + 4k)) per cut face, and 28 k^3 per
    ghost-penalty derivative order and face.
    """
    k = p + 1
    nd = k**dim
    seg = info["seg"]
    n_vol = seg[2] - seg[1]
    n_fcut = seg[4] - seg[3]
    n_surf = seg[5] - seg[4]
    b = {
        "structured": (info["n_inside"] + info["n_cut"]) * nd * 2 * s,
        "cut_lines": info["n_cut"] * nd * 3 * s + n_vol * (dim + 1) * s + n_surf * (2 * dim + 1) * s,
        "cut_face_lines": info["n_cut"] * nd * 3 * s + n_fcut * dim * s,
    }
    # the whole apply: u read and v written once per DoF, plus the point data
    b["total"] = info["n_dofs"] * 2 * s + n_vol * (dim + 1) * s + n_surf * (2 * dim + 1) * s + n_fcut * dim * s
    if mixed:
        # the element matrices replace the volume and interface point data
        mat = info["n_cut"] * nd * nd * s
        b["cut_lines"] = info["n_cut"] * nd * 3 * s + mat
        b["total"] += mat - n_vol * (dim + 1) * s - n_surf * (2 * dim + 1) * s
    if kappa:
        k_str = (seg[1] - seg[0]) + (seg[3] - seg[2])
        b["structured"] += k_str * s
        b["cut_lines"] += (n_vol + n_surf) * s
        b["cut_face_lines"] += n_fcut * s
        b["total"] += info["n_qp"] * s
    flops = None
    if dim == 3:
        flops = (
            info["n_inside"] * 24 * k**4
            + info["n_faces_str"] * 56 * k**3
            + info["n_faces_gp"] * 28 * k**3 * (p + 1)
            + (n_vol + n_surf) * 4 * (2 * k**3 + 3 * k**2 + 4 * k)
            + 8 * (info["n_faces_cut"] * k**3 + n_fcut * (3 * k**2 + 4 * k))
        )
    return b, flops


def load_counters(kernel_key):
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    ent = data.get(kernel_key)
    if not ent or ent.get("kernel_hash") != kernel_hash():
        return None
    return ent


WORKLOADS = {
    "ball3d": lambda seed, n, degree: __import__("ufem_inputs").ball3d(seed, n=n or 64, degree=degree or 3),
    "kappa3d": lambda seed, n, degree: __import__("ufem_inputs").kappa3d(seed, n=n or 48, degree=degree or 4),
    "balls3d": lambda seed, n, degree: __import__("ufem_inputs").balls3d(seed, n=n or 128, degree=degree or 3),
    "sweep3d": lambda seed, n, degree: __import__("ufem_inputs").sweep3d(degree or 3, seed, n=n),
    "disk2d": lambda seed, n, degree: __import__("ufem_inputs").disk2d(seed, n=n or 16, degree=degree or 2),
}


def make_workload(name, seed, n=None, degree=None, layer=None):
    import ufem_inputs as ui

    if name == "plane3d":
        return ui.plane3d(layer if layer is not None else 1, seed, n=n or 128, degree=degree or 1)
    return WORKLOADS[name](seed, n, degree)


def _oracle(wl):
    from oracle.operator import UnfittedDG

    return UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, wl.lo, wl.hi, plane=wl.plane)


def _prepare_rules(ora, cells):
    """quadrature generation is setup, not timed"""
    cellset = set(int(b) for b in cells)
    for b in cellset:
        if ora.cls[b] == 1:
            ora.cell_rule(b)
    for fi, f in enumerate(ora.faces):
        if f[3] == "cut" and (f[0] in cellset or f[1] in cellset):
            ora.face_rule(fi)


def _oracle_worker(spec):
    """One process of the all-cores oracle run: the workload's oracle, the
    seeded u, its share of the sampled cells; times the apply on them once
    every worker is ready."""
    import numpy as np

    import ufem_inputs as ui

    wl, rng = make_workload(spec["workload"], spec["seed"], spec["n"], spec["degree"], spec["layer"])
    ora = _oracle(wl)
    u = ui.uniform_vector(rng, ora.n_dofs)
    cells = spec["cells"]
    _prepare_rules(ora, cells)
    spec["barrier"].wait()
    t0 = time.perf_counter()
    v = ora.apply(u, cells=cells)
    dt = time.perf_counter() - t0
    rows = np.concatenate([v[ora.rank[b] * ora.nd:(ora.rank[b] + 1) * ora.nd] for b in cells]) if cells else v[:0]
    return len(cells) * ora.nd, dt, rows


def cpu_baseline(args, wl, u, seconds_target=12.0, seed=1234):
    """The FP64 oracle, as it stands, on bounded samples of the same
    workload's rows (cells in the workload's inside / cut proportion): on one
    core in this process, then on every core the process may use (at most
    16), one oracle process per core, each on its share of a larger sample.
    Returns the baseline record and the oracle rows of the one-core sample."""
    import multiprocessing as mp

    import numpy as np

    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None

    ora = _oracle(wl)
    rng = np.random.default_rng(seed)
    n_in, n_cut = len(ora.inside_cells), len(ora.cut_cells)
    frac_cut = n_cut / max(1, n_in + n_cut)

    def sample(n_sample):
        nc = min(n_cut, max(1 if n_cut else 0, int(round(n_sample * frac_cut))))
        ni = min(n_in, max(0, n_sample - nc))
        return [int(b) for b in rng.choice(ora.inside_cells, ni, replace=False)] + [
            int(b) for b in rng.choice(ora.cut_cells, nc, replace=False)]

    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        probe = sample(24)
        _prepare_rules(ora, probe)
        ora.apply(u, cells=probe)
        t0 = time.perf_counter()
        ora.apply(u, cells=probe)
        per_cell = (time.perf_counter() - t0) / len(probe)
        cells1 = sample(int(max(24, min(n_in + n_cut, seconds_target / max(per_cell, 1e-6)))))
        _prepare_rules(ora, cells1)
        t0 = time.perf_counter()
        v1 = ora.apply(u, cells=cells1)
        dt1 = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    dofs1 = len(cells1) * ora.nd
    n1i = sum(1 for b in cells1 if ora.cls[b] == 0)
    one = {"value": dofs1 / dt1, "unit": "DoF/s", "cores": 1,
           "sample": f"rows of {len(cells1)} of {n_in + n_cut} active cells ({n1i} inside, {len(cells1) - n1i} cut, "
                     f"seeded), {dofs1} DoF, {dt1:.1f} s, one thread (BLAS limited to 1)"}
    out = dict(one, kind="oracle")
    cores = min(len(os.sched_getaffinity(0)), 16)
    progress(f"oracle on one core: {one['value']:.3g} DoF/s")
    if cores > 1 and not args.cpu_one_core:
        progress(f"oracle on {cores} cores")
        per_worker = int(max(24, seconds_target / max(dt1 / len(cells1), 1e-6)))
        cells_all = sample(min(n_in + n_cut, per_worker * cores))
        chunks = [cells_all[i::cores] for i in range(cores)]
        saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
        for k in saved:
            os.environ[k] = "1"
        try:
            sp = mp.get_context("spawn")
            with sp.Manager() as mgr:
                barrier = mgr.Barrier(cores)
                specs = [{"workload": wl.name if wl.name != "custom" else "ball3d", "seed": args.seed, "n": args.n,
                          "degree": args.degree, "layer": args.layer, "cells": c, "barrier": barrier} for c in chunks]
                with sp.Pool(cores) as pool:
                    res = pool.map(_oracle_worker, specs)
        finally:
            for k, val in saved.items():
                if val is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = val
        dofs = sum(r[0] for r in res)
        dt = max(r[1] for r in res)
        ni = sum(1 for b in cells_all if ora.cls[b] == 0)
        out = {"value": dofs / dt, "unit": "DoF/s", "cores": cores, "kind": "oracle",
               "sample": f"rows of {len(cells_all)} of {n_in + n_cut} active cells ({ni} inside, "
                         f"{len(cells_all) - ni} cut, seeded), {dofs} DoF, {cores} oracle processes of one "
                         f"thread each (BLAS limited to 1), {dt:.1f} s for the slowest",
               "single_core": one}
    rows1 = (cells1, np.concatenate([v1[ora.rank[b] * ora.nd:(ora.rank[b] + 1) * ora.nd] for b in cells1]), ora)
    return out, rows1


def oracle_errors(wl, info, cls, v64, v32, atw, dk, rows1):
    """Largest error against the FP64 oracle relative to the largest oracle
    entry, on sampled rows: the stored oracle rows of the full-size
    workloads (tests/golden, written by the oracle for the same seeded
    inputs) when they match this workload, else the rows of the one-core
    oracle sample (FP64 apply only).  v64, v32, atw, dk: host arrays."""
    import numpy as np

    nd = (wl.degree + 1) ** wl.dim
    tag = f"sweep{wl.degree}" if wl.name == "sweep3d" else wl.name
    path = os.path.join(ROOT, "tests", "golden", f"fullsize_{tag}.npz")
    rank = np.cumsum(cls != 2) - 1

    def err(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())

    def rows(v, cells):
        return np.stack([v[rank[b] * nd:(rank[b] + 1) * nd] for b in cells])

    if os.path.exists(path):
        ref = np.load(path)
        if int(ref["n_dofs"]) == info["n_dofs"] and int(ref["degree"]) == wl.degree and int(ref["n"]) == wl.n:
            cells = [int(b) for b in ref["cells"]]
            out = {"fp64_apply": err(rows(v64, cells), ref["rows64"]),
                   "fp32_apply": err(rows(v32, cells), ref["rows32"]),
                   "adjoint_ATw": err(rows(atw, cells), ref["rows_adj"])}
            if "dk_idx" in ref and dk is not None:
                out["adjoint_dkappa"] = err(dk[ref["dk_idx"]], ref["dk_val"])
            out["rows"] = f"{len(cells)} sampled cells, stored oracle rows (tests/golden/fullsize_{tag}.npz)"
            return out
    if rows1 is not None:
        cells, ref_rows, _ = rows1
        return {"fp64_apply": err(rows(v64, cells).reshape(-1), ref_rows),
                "rows": f"{len(cells)} cells of the one-core oracle sample"}
    return None


def run_solve(op, plan, rng, tol, inner_rtol):
    """A u = b with b = A u*, u* uniform in [-1, 1]: plain FP64 CG against
    FP32-inner / FP64-outer defect correction, both to ||b - A u|| <= tol ||b||
    measured in FP64 on the GPU."""
    import torch

    import ufem_inputs as ui
    from paper_2404_07911_amd.solvers import DeviceOps, device_cg, device_defect_correction, device_reliable_cg, timed

    ops = DeviceOps(0)
    n = plan.info["n_dofs"]
    ustar = torch.from_numpy(ui.uniform_vector(rng, n)).cuda()
    b = op.apply(ustar)
    x = torch.zeros_like(b)
    last = [time.perf_counter()]

    def tick(it, res):
        # a progress line at most every 20 s (long solves stay visibly alive)
        if time.perf_counter() - last[0] > 20.0:
            last[0] = time.perf_counter()
            progress(f"solve: {it} iterations, relative residual {res:.2e}")

    (x, i64), t64 = timed(lambda: device_cg(op, b, x, rtol=tol, maxiter=400000, progress=tick), ops)
    r = op.apply(x)
    res64 = float(torch.linalg.norm(b - r) / torch.linalg.norm(b))
    progress(f"solve: FP64 CG done ({i64['iterations']} iterations, {t64:.1f} s); defect correction")
    (u, idc), tdc = timed(lambda: device_defect_correction(op, b, tol=tol, inner_rtol=inner_rtol, progress=tick), ops)
    r = op.apply(u)
    resdc = float(torch.linalg.norm(b - r) / torch.linalg.norm(b))
    progress(f"solve: defect correction done ({idc['inner_iterations']} inner iterations, {tdc:.1f} s); "
             "FP32 CG with reliable updates")
    (u2, irl), trl = timed(lambda: device_reliable_cg(op, b, tol=tol, progress=tick), ops)
    resrl = float(torch.linalg.norm(b - op.apply(u2)) / torch.linalg.norm(b))
    err = float(torch.linalg.norm(u - ustar) / torch.linalg.norm(ustar))
    w = (r - b).contiguous()
    atw = torch.empty_like(w)
    dk = torch.empty(plan.info["n_qp"], dtype=torch.float64, device=w.device)
    (_, tadj) = timed(lambda: op.apply_adjoint(w, u, atw, dk), ops)
    return {
        "tol": tol,
        "speedup_fp32_inner_over_fp64": t64 / tdc,
        "fp64_cg": {"seconds": t64, "iterations": i64["iterations"], "rel_residual": res64,
                    "converged": i64["converged"]},
        "defect_correction": {"seconds": tdc, "outer": idc["outer"], "inner_iterations": idc["inner_iterations"],
                              "rel_residual": resdc, "converged": idc["converged"], "inner_rtol": inner_rtol},
        "reliable_update_cg": {"seconds": trl, "fp32_iterations": irl["iterations"], "updates": irl["updates"],
                               "rel_residual": resrl, "converged": irl["converged"],
                               "speedup_over_fp64": t64 / trl},
        "solution_rel_error": err,
        "adjoint_at_solution_s": tadj,
    }


def workload_text(wl, space="dg", gp="face"):
    if wl.plane is not None:
        geo = f"plane n={list(np.round(wl.plane[0], 6))} offset {wl.plane[1]:.6f}"
    else:
        geo = f"{len(wl.radii)} ball(s)"
    disc = "SIPG DG" if space == "dg" else "continuous FE_Q"
    gpt = {"face": "face ghost penalty", "volume": "volume ghost penalty (stable neighbours)",
           "volume_all": "volume ghost penalty (all neighbours)"}[gp]
    return (f"{wl.name}: {wl.dim}D {disc} p={wl.degree}, {wl.n}^{wl.dim} background cells on [-1,1]^{wl.dim}, "
            f"{geo}, Nitsche + {gpt}" + (", kappa field" if wl.name == "kappa3d" else ""))


def solve_mode(args, wl, rng, plan, op, t_setup):
    """--mode solve: the solve comparison of run_solve as its own line."""
    n = plan.info["n_dofs"]
    sol = run_solve(op, plan, rng, args.tol, args.inner_rtol)
    out = {
        "metric": "solve time to 1e-10 relative residual, FP64 CG vs FP32-inner defect correction",
        "value": sol["speedup_fp32_inner_over_fp64"],
        "unit": "speedup",
        "higher_is_better": True,
        "n_gpus": 1,
        "dtype": "f64/f32",
        "data": "synthetic",
        "config": {"workload": workload_text(wl), "active_dofs": n, "degree": wl.degree, "background_cells": wl.n},
        **{k: v for k, v in sol.items() if k != "speedup_fp32_inner_over_fp64"},
        "setup_s": t_setup,
        "kernel_hash": kernel_hash(),
    }
    print(json.dumps(out), flush=True)
    return 0


def plane_sweep_mode(args):
    """Throughput against the ratio of cut to physical cells (the plane
    benchmark, Section 5.2): the domain below a plane in cell layer L of an
    n^3 mesh (ratio 1 / (L + 1); no cut cell for L >= n), FP64 and FP32
    applies timed with HIP events, vectors resident in HBM."""
    import torch

    import ufem_inputs as ui
    from paper_2404_07911_amd import Operator, Plan, Problem

    n = args.n or 128
    degrees = [args.degree] if args.degree else [1, 3]
    layers = [0, 1, 9, 99, n]
    stream = torch.cuda.current_stream()
    points = []
    for p in degrees:
        for layer in layers:
            wl, rng = ui.plane3d(layer, args.seed, n=n, degree=p)
            plan = Plan(Problem.from_workload(wl))
            op = Operator(plan, device=0)
            info = plan.info
            nd = info["n_dofs"]
            u = torch.from_numpy(ui.uniform_vector(rng, nd)).cuda()
            rec = {"degree": p, "layer": layer, "active_cells": info["n_active"], "cut_cells": info["n_cut"],
                   "cut_cell_ratio": info["n_cut"] / max(1, info["n_active"]), "active_dofs": nd}
            for name, x in (("fp64", u), ("fp32", u.to(torch.float32))):
                pairs = max(2, int(math.ceil(args.cache_bytes / (2 * x.element_size() * nd))))
                X = [x.clone() for _ in range(pairs)]
                V = [torch.empty_like(x) for _ in range(pairs)]
                for i in range(args.warmup):
                    op.apply(X[i % pairs], V[i % pairs])
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(args.steps)]
                torch.cuda.synchronize()
                for i in range(args.steps):
                    ev[i][0].record(stream)
                    op.apply(X[i % pairs], V[i % pairs])
                    ev[i][1].record(stream)
                torch.cuda.synchronize()
                ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
                rec[f"{name}_apply_ms"] = ms
                rec[f"{name}_dofs_per_s"] = nd / (ms * 1e-3)
                del X, V
            print(f"plane sweep p={p} layer={layer}: ratio {rec['cut_cell_ratio']:.3f}, {nd} DoF, "
                  f"FP64 {rec['fp64_dofs_per_s'] / 1e9:.1f} GDoF/s", file=sys.stderr, flush=True)
            points.append(rec)
            del op, plan, u
            torch.cuda.empty_cache()
    out = {
        "metric": "operator DoF/s against the cut-cell ratio (plane benchmark)",
        "value": None,
        "unit": "DoF/s",
        "higher_is_better": True,
        "n_gpus": 1,
        "dtype": "f64/f32",
        "data": "synthetic",
        "config": {"workload": f"plane3d: 3D SIPG DG, {n}^3 background cells on [-1,1]^3, domain below a plane "
                               f"z ~ const (normal tilted by {ui.PLANE_TILT}) in cell layer L, "
                               f"Nitsche + face ghost penalty", "background_cells": n},
        "points": points,
        "kernel_hash": kernel_hash(),
    }
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ball3d",
                    choices=["ball3d", "kappa3d", "balls3d", "sweep3d", "disk2d", "plane3d"])
    ap.add_argument("--degree", type=int, default=None)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--layer", type=int, default=None,
                    help="plane3d: cell layer of the plane (cut-cell ratio 1 / (layer + 1); >= n: no cut)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cache-bytes", type=float, default=640e6, help="total bytes of rotated vector pairs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-one-core", action="store_true", help="oracle baseline on one core only")
    ap.add_argument("--no-solve", action="store_true", help="skip the solve comparison of the default line")
    ap.add_argument("--space", default="dg", choices=["dg", "cg"],
                    help="dg: SIPG discontinuous space (default); cg: continuous FE_Q space")
    ap.add_argument("--gp", default="face", choices=["face", "volume", "volume_all"],
                    help="ghost penalty: face (default), volume (stable neighbours), volume_all")
    ap.add_argument("--mixed", action="store_true",
                    help="mixed evaluation: the cut cells' volume and interface terms as precomputed element matrices")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--mode", default="apply", choices=["apply", "solve", "plane-sweep"],
                    help="apply: operator throughput (default); solve: FP64 CG vs FP32-inner defect correction; "
                         "plane-sweep: throughput against the cut-cell ratio (plane benchmark)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--inner-rtol", type=float, default=1e-4)
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(
            "bench.py measures one GPU only: the operator has no multi-GPU path "
            "(each GPU would own a block of cells and exchange a halo of face data); run with --gpus 1",
            file=sys.stderr,
        )
        return 2

    import torch

    import ufem_inputs as ui
    from paper_2404_07911_amd import Operator, Plan, Problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.mode == "plane-sweep":
        return plane_sweep_mode(args)

    wl, rng = make_workload(args.workload, args.seed, args.n, args.degree, args.layer)

    progress(f"plan and setup of {wl.name} p={wl.degree} n={wl.n} ({args.space}, {args.gp} ghost penalty)")
    t0 = time.perf_counter()
    plan = Plan(Problem.from_workload(wl, space=args.space, gp_kind=args.gp))
    op = Operator(plan, device=0)
    t_setup = time.perf_counter() - t0
    info = plan.info
    n = info["n_dofs"]
    with_kappa = wl.name == "kappa3d"
    if with_kappa:
        # variable coefficient at every quadrature point (the kappa workload)
        op.set_kappa(torch.from_numpy(ui.kappa_field(plan.qp()[0])).to(dev))
    if args.mixed:
        progress("element matrices of the cut cells (mixed evaluation)")
        t0 = time.perf_counter()
        op.set_mixed(True)
        t_setup += time.perf_counter() - t0
    if args.mode == "solve":
        return solve_mode(args, wl, rng, plan, op, t_setup)
    u_host = ui.uniform_vector(rng, n)
    w_host = ui.uniform_vector(rng, n)

    npairs = max(2, int(math.ceil(args.cache_bytes / (2 * 8 * n))))
    U64 = [torch.from_numpy(u_host).to(dev) if i == 0 else torch.empty(n, dtype=torch.float64, device=dev) for i in range(npairs)]
    for i in range(1, npairs):
        U64[i].copy_(U64[0])
    V64 = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(npairs)]
    U32 = [x.to(torch.float32) for x in U64]
    V32 = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(npairs)]
    W64 = torch.from_numpy(w_host).to(dev)
    ATW = torch.empty(n, dtype=torch.float64, device=dev)
    DK = torch.empty(info["n_qp"], dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    # one step: the FP64 apply and the FP32 apply stage by stage (each stage
    # one kernel, bracketed by events on the library's stream), then the FP64
    # adjoint pass
    NS = len(STAGES)
    NEV = 2 * NS + 2

    def step(i, ev=None):
        j = i % npairs
        k = 0
        for U, V in ((U64[j], V64[j]), (U32[j], V32[j])):
            for part in STAGES:
                if ev is not None:
                    ev[k].record(stream)
                k += 1
                if args.space == "cg":
                    # the continuous space applies every stage at once (node
                    # gather and sums around the cell kernels): timed whole
                    if part == 3:
                        op.apply(U, V)
                else:
                    op.apply_part(part, U, V)
        if ev is not None:
            ev[2 * NS].record(stream)
        op.apply_adjoint(W64, U64[j], ATW, DK)
        if ev is not None:
            ev[2 * NS + 1].record(stream)

    progress("warmup and timed steps")
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(NEV)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i, evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    def mean_ms(a, b):
        return float(np.mean([e[a].elapsed_time(e[b]) for e in evs]))

    names = list(STAGES.values())
    ms64 = {nm: mean_ms(q, q + 1) for q, nm in enumerate(names)}
    ms32 = {nm: mean_ms(NS + q, NS + q + 1) for q, nm in enumerate(names)}
    adj = mean_ms(2 * NS, 2 * NS + 1)
    step_ms = mean_ms(0, 2 * NS + 1)
    t64 = mean_ms(0, NS) * 1e-3
    t32 = mean_ms(NS, 2 * NS) * 1e-3
    tadj = adj * 1e-3

    # the results of the timed configuration on the first pair, for the
    # error against the oracle
    v64_h = op.apply(U64[0]).cpu().numpy()
    v32_h = op.apply(U32[0]).cpu().numpy().astype(np.float64)
    op.apply_adjoint(W64, U64[0], ATW, DK)
    atw_h, dk_h = ATW.cpu().numpy(), DK.cpu().numpy()
    assert np.isfinite(v64_h).all() and np.isfinite(v32_h).all() and np.isfinite(atw_h).all()
    if not args.no_solve:
        progress("solve: FP64 CG and FP32-inner defect correction")
    sol = None if args.no_solve else run_solve(op, plan, rng, args.tol, args.inner_rtol)

    bytes64, flops = model(info, wl.dim, wl.degree, 8, with_kappa, args.mixed)
    bytes32, _ = model(info, wl.dim, wl.degree, 4, with_kappa, args.mixed)
    dom = max(ms64, key=ms64.get)
    dom_ms = ms64[dom]
    achieved = bytes64[dom] / (dom_ms * 1e-3) / 1e9
    if args.space == "cg":
        # one timed launch sequence per apply: the whole apply is the unit
        dom, dom_ms = "total", t64 * 1e3
        achieved = bytes64["total"] / t64 / 1e9
    ctr = load_counters(f"{args.workload}_p{wl.degree}_n{wl.n}_{dom}_f64")
    traffic = ctr["hbm_bytes_per_launch"] if ctr else None
    roofline = {
        "bound": "hbm",
        "kernel": ("whole apply of the continuous space (node gather, cell kernels, node sums)" if dom == "total"
                   else f"{(STAGE_KERNELS_MIXED if args.mixed else STAGE_KERNELS)[dom]}")
        + f", K={wl.degree + 1}, D={wl.dim}, double",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "algorithmic_bytes_per_launch": bytes64[dom],
        "launch_ms": dom_ms,
    }
    apply_gbs = bytes64["total"] / t64 / 1e9
    out = {
        "metric": METRIC,
        "value": n / t64,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": workload_text(wl, args.space, args.gp),
            "degree": wl.degree,
            "background_cells": wl.n,
            "active_dofs": n,
            "background_dofs": info["n_background"] * (wl.degree + 1) ** wl.dim,
            "kappa": "1 + 0.5 sin(pi x) sin(pi y) sin(pi z) per quadrature point" if with_kappa else "1",
            "inside_cells": info["n_inside"],
            "cut_cells": info["n_cut"],
            "cut_cell_ratio": info["n_cut"] / max(1, info["n_active"]),
            "evaluation": "mixed (cut-cell volume and interface terms as element matrices)" if args.mixed
            else "matrix-free",
            "space": "continuous Q_p (FE_Q), Poisson + Nitsche" if args.space == "cg" else "discontinuous Q_p, SIPG",
            "ghost_penalty": args.gp,
            "cell_dofs": info["n_cell_dofs"],
            "quadrature_points": info["n_qp"],
            "parallelism": "single GPU",
        },
        "fp64_apply_ms": t64 * 1e3,
        "fp32_value": n / t32,
        "fp32_apply_ms": t32 * 1e3,
        "fp32_speedup": t64 / t32,
        "adjoint_value": n / tadj,
        "adjoint_ms": tadj * 1e3,
        "kernels_ms": {**{f"{nm}_f64": ms64[nm] for nm in names}, **{f"{nm}_f32": ms32[nm] for nm in names},
                       "adjoint_f64": adj},
        "kernels_hbm_frac_f64": ({nm: bytes64[nm] / (ms64[nm] * 1e-3) / 1e9 / HBM_PEAK_GBS for nm in names}
                                 if args.space == "dg" else None),
        "apply_hbm_frac_f64": apply_gbs / HBM_PEAK_GBS,
        "apply_hbm_frac_f32": bytes32["total"] / t32 / 1e9 / HBM_PEAK_GBS,
        "model_gflop_per_apply": flops / 1e9 if flops else None,
        "alu_frac_f64": (flops / t64 / 1e12 / FP64_PEAK_TFLOPS) if flops else None,
        "roofline": roofline,
        "setup_s": t_setup,
        "wall_s_timed": wall,
        "rotated_pairs": npairs,
        "kernel_hash": kernel_hash(),
    }
    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.copy_(a)
        e1.record(stream)
        torch.cuda.synchronize()
        out["copy_probe"] = {"bytes_read": a.numel() * 8, "ms": e0.elapsed_time(e1),
                             "gbs": 2 * a.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9}
    rows1 = None
    if args.space == "cg" or args.gp != "face":
        args.no_cpu_baseline = True  # the baseline and the stored rows are the default discretisation's
    if not args.no_cpu_baseline:
        progress("oracle baseline on the host cores")
        out["cpu_baseline"], rows1 = cpu_baseline(args, wl, u_host, args.cpu_seconds)
        out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
    out["error_vs_oracle"] = (oracle_errors(wl, info, plan.cells(), v64_h, v32_h, atw_h, dk_h, rows1)
                              if args.space == "dg" and args.gp == "face" else None)
    if sol is not None:
        out["solve"] = sol
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
