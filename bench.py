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
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "operator DoF/s (3D DG k=3, FP64 vs FP32) + adjoint DoF/s; % of HBM roofline"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64, published
KERNEL_SOURCES = ["paper_2404_07911_amd/csrc/kernels_impl.hpp", "paper_2404_07911_amd/csrc/device.hpp"]


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


def model(info, dim, p, s, kappa=False):
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


def cpu_baseline(wl, u, seconds_target=15.0, seed=1234):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    workload's rows (cells in the workload's inside/cut proportion)."""
    import numpy as np

    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle.operator import UnfittedDG

    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        ora = UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii, wl.lo, wl.hi)
        rng = np.random.default_rng(seed)
        n_in, n_cut = len(ora.inside_cells), len(ora.cut_cells)
        frac_cut = n_cut / max(1, n_in + n_cut)
        # probe the per-cell cost, then size the sample to ~seconds_target
        probe = list(rng.choice(ora.inside_cells, 20, replace=False)) + list(rng.choice(ora.cut_cells, 4, replace=False))
        ora.apply(u, cells=probe)
        t0 = time.perf_counter()
        ora.apply(u, cells=probe)
        per_cell = (time.perf_counter() - t0) / len(probe)
        n_sample = int(max(24, min(n_in + n_cut, seconds_target / max(per_cell, 1e-6))))
        nc = max(1, int(round(n_sample * frac_cut)))
        ni = max(1, n_sample - nc)
        cells = list(rng.choice(ora.inside_cells, min(ni, n_in), replace=False)) + list(
            rng.choice(ora.cut_cells, min(nc, n_cut), replace=False)
        )
        cellset = set(int(b) for b in cells)
        for b in cellset:  # quadrature generation is setup, not timed
            if ora.cls[b] == 1:
                ora.cell_rule(b)
        for fi, f in enumerate(ora.faces):
            if f[3] == "cut" and (f[0] in cellset or f[1] in cellset):
                ora.face_rule(fi)
        t0 = time.perf_counter()
        ora.apply(u, cells=cells)
        dt = time.perf_counter() - t0
        dofs = len(cells) * ora.nd
        return {
            "value": dofs / dt,
            "unit": "DoF/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"rows of {len(cells)} of {n_in + n_cut} active cells ({len(cells) - min(nc, n_cut)} inside, "
            f"{min(nc, n_cut)} cut, seeded), {dofs} DoF, {dt:.1f} s, one thread (BLAS limited to 1)",
        }
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)


def solve_mode(args, wl, rng, plan, op, t_setup):
    """A u = b with b = A u*, u* uniform in [-1, 1]: plain FP64 CG against
    FP32-inner / FP64-outer defect correction, both to ||b - A u|| <= tol ||b||
    measured in FP64 on the GPU."""
    import torch

    import ufem_inputs as ui
    from paper_2404_07911_amd.solvers import DeviceOps, device_cg, device_defect_correction, timed

    ops = DeviceOps(0)
    n = plan.info["n_dofs"]
    ustar = torch.from_numpy(ui.uniform_vector(rng, n)).cuda()
    b = op.apply(ustar)

    x = torch.zeros_like(b)
    (x, i64), t64 = timed(lambda: device_cg(op, b, x, rtol=args.tol, maxiter=400000), ops)
    r = op.apply(x)
    res64 = float(torch.linalg.norm(b - r) / torch.linalg.norm(b))
    (u, idc), tdc = timed(lambda: device_defect_correction(op, b, tol=args.tol, inner_rtol=args.inner_rtol), ops)
    r = op.apply(u)
    resdc = float(torch.linalg.norm(b - r) / torch.linalg.norm(b))
    err = float(torch.linalg.norm(u - ustar) / torch.linalg.norm(ustar))
    # one adjoint pass at the solution: A^T w and dL/dkappa for w = A u - b
    w = (r - b).contiguous()
    atw = torch.empty_like(w)
    dk = torch.empty(plan.info["n_qp"], dtype=torch.float64, device=w.device)
    (_, tadj) = timed(lambda: op.apply_adjoint(w, u, atw, dk), ops)
    out = {
        "metric": "solve time to 1e-10 relative residual, FP64 CG vs FP32-inner defect correction",
        "value": t64 / tdc,
        "unit": "speedup",
        "higher_is_better": True,
        "n_gpus": 1,
        "dtype": "f64/f32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.dim}D SIPG DG p={wl.degree}, {wl.n}^{wl.dim} background cells, "
                               f"{len(wl.radii)} ball(s)" + (", kappa field" if wl.name == "kappa3d" else ""),
                   "active_dofs": n, "degree": wl.degree, "background_cells": wl.n},
        "fp64_cg": {"seconds": t64, "iterations": i64["iterations"], "rel_residual": res64,
                    "converged": i64["converged"]},
        "defect_correction": {"seconds": tdc, "outer": idc["outer"], "inner_iterations": idc["inner_iterations"],
                              "rel_residual": resdc, "converged": idc["converged"], "history": idc["history"],
                              "inner_rtol": args.inner_rtol},
        "solution_rel_error": err,
        "adjoint_at_solution_s": tadj,
        "setup_s": t_setup,
        "kernel_hash": kernel_hash(),
    }
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ball3d", choices=["ball3d", "kappa3d", "balls3d", "sweep3d", "disk2d"])
    ap.add_argument("--degree", type=int, default=None)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cache-bytes", type=float, default=640e6, help="total bytes of rotated vector pairs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--mode", default="apply", choices=["apply", "solve"],
                    help="apply: operator throughput (default); solve: FP64 CG vs FP32-inner defect correction")
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

    import numpy as np
    import torch

    import ufem_inputs as ui
    from paper_2404_07911_amd import Operator, Plan, Problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.workload == "ball3d":
        wl, rng = ui.ball3d(args.seed, n=args.n or 64, degree=args.degree or 3)
    elif args.workload == "kappa3d":
        wl, rng = ui.kappa3d(args.seed, n=args.n or 48, degree=args.degree or 4)
    elif args.workload == "balls3d":
        wl, rng = ui.balls3d(args.seed, n=args.n or 128, degree=args.degree or 3)
    elif args.workload == "sweep3d":
        wl, rng = ui.sweep3d(args.degree or 3, args.seed, n=args.n)
    else:
        wl, rng = ui.disk2d(args.seed, n=args.n or 16, degree=args.degree or 2)

    t0 = time.perf_counter()
    plan = Plan(Problem.from_workload(wl))
    op = Operator(plan, device=0)
    t_setup = time.perf_counter() - t0
    info = plan.info
    n = info["n_dofs"]
    with_kappa = wl.name == "kappa3d"
    if with_kappa:
        # variable coefficient at every quadrature point (the kappa workload)
        op.set_kappa(torch.from_numpy(ui.kappa_field(plan.qp()[0])).to(dev))
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
                op.apply_part(part, U, V)
        if ev is not None:
            ev[2 * NS].record(stream)
        op.apply_adjoint(W64, U64[j], ATW, DK)
        if ev is not None:
            ev[2 * NS + 1].record(stream)

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

    # correctness spot check of the timed FP64 result against a fresh apply
    vchk = op.apply(U64[0])
    torch.cuda.synchronize()
    assert torch.isfinite(vchk).all()

    bytes64, flops = model(info, wl.dim, wl.degree, 8, with_kappa)
    bytes32, _ = model(info, wl.dim, wl.degree, 4, with_kappa)
    dom = max(ms64, key=ms64.get)
    dom_ms = ms64[dom]
    achieved = bytes64[dom] / (dom_ms * 1e-3) / 1e9
    ctr = load_counters(f"{args.workload}_p{wl.degree}_n{wl.n}_{dom}_f64")
    traffic = ctr["hbm_bytes_per_launch"] if ctr else None
    roofline = {
        "bound": "hbm",
        "kernel": f"{STAGE_KERNELS[dom]}, K={wl.degree + 1}, D={wl.dim}, double",
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
            "workload": f"{wl.name}: {wl.dim}D SIPG DG p={wl.degree}, {wl.n}^{wl.dim} background cells on [-1,1]^{wl.dim}, "
            f"{len(wl.radii)} ball(s), Nitsche + face ghost penalty",
            "degree": wl.degree,
            "background_cells": wl.n,
            "active_dofs": n,
            "background_dofs": info["n_background"] * (wl.degree + 1) ** wl.dim,
            "kappa": "1 + 0.5 sin(pi x) sin(pi y) sin(pi z) per quadrature point" if with_kappa else "1",
            "inside_cells": info["n_inside"],
            "cut_cells": info["n_cut"],
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
        "kernels_hbm_frac_f64": {nm: bytes64[nm] / (ms64[nm] * 1e-3) / 1e9 / HBM_PEAK_GBS for nm in names},
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
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, u_host, args.cpu_seconds)
        out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
