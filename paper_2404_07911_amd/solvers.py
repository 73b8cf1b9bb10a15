"""Iterative solvers around the operator: conjugate gradients, the
mixed-precision defect correction (FP32 inner solves, FP64 residual and
update) and FP32 CG with FP64 reliable updates (residual replacement),
written against a small vector-operations interface or the device CG of
libufem.

The paper solves with a preconditioned CG (Section 3.6); the
preconditioners it uses live in external libraries and are not part of
this package, so the drivers here are unpreconditioned.

`DeviceOps` runs every vector operation in the HIP BLAS-1 kernels of
libufem (dot products accumulate in float64 for both precisions and come
back to the host as one scalar per call).  The drivers accept any apply
callable and any ops object with the same methods.
"""
from __future__ import annotations

import ctypes as C
import math
import time

from . import _lib as L


class DeviceOps:
    """Vector operations on device tensors through the C ABI."""

    def __init__(self, device: int = 0):
        import torch

        self.torch = torch
        self.device = torch.device(f"cuda:{device}")
        self._scalar = torch.zeros(1, dtype=torch.float64, device=self.device)

    @staticmethod
    def _prec(t):
        import torch

        return L.F64 if t.dtype == torch.float64 else L.F32

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def dot(self, x, y) -> float:
        L.check(L.lib().ufem_dot(self._prec(x), x.numel(), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                 C.c_void_p(self._scalar.data_ptr()), self._stream()))
        return float(self._scalar.item())

    def axpby(self, a, x, b, y):
        """y = a x + b y (in place)."""
        L.check(L.lib().ufem_axpby(self._prec(y), y.numel(), float(a), C.c_void_p(x.data_ptr()), float(b),
                                   C.c_void_p(y.data_ptr()), self._stream()))
        return y

    def copy(self, dst, src):
        L.check(L.lib().ufem_cast(self._prec(src), self._prec(dst), src.numel(), C.c_void_p(src.data_ptr()),
                                  C.c_void_p(dst.data_ptr()), self._stream()))
        return dst

    def cast(self, x, dtype):
        out = self.torch.empty(x.numel(), dtype=dtype, device=x.device)
        return self.copy(out, x)

    def zeros_like(self, x, dtype=None):
        return self.torch.zeros(x.numel(), dtype=dtype or x.dtype, device=x.device)

    def empty_like(self, x, dtype=None):
        return self.torch.empty(x.numel(), dtype=dtype or x.dtype, device=x.device)

    def f32(self):
        return self.torch.float32

    def f64(self):
        return self.torch.float64

    def sync(self):
        self.torch.cuda.synchronize()


class HostOps:
    """The same interface on numpy arrays (for the solver logic on the CPU)."""

    def __init__(self):
        import numpy as np

        self.np = np

    def dot(self, x, y) -> float:
        return float(self.np.dot(x.astype(self.np.float64), y.astype(self.np.float64)))

    def axpby(self, a, x, b, y):
        y[:] = (a * x.astype(self.np.float64) + b * y.astype(self.np.float64)).astype(y.dtype)
        return y

    def copy(self, dst, src):
        dst[:] = src.astype(dst.dtype)
        return dst

    def cast(self, x, dtype):
        return x.astype(dtype)

    def zeros_like(self, x, dtype=None):
        return self.np.zeros(x.size, dtype=dtype or x.dtype)

    def empty_like(self, x, dtype=None):
        return self.np.empty(x.size, dtype=dtype or x.dtype)

    def f32(self):
        return self.np.float32

    def f64(self):
        return self.np.float64

    def sync(self):
        pass


def cg(apply, b, x, ops, rtol=1e-10, maxiter=10000, rnorm0=None):
    """Unpreconditioned CG for the SPD operator `apply`; x is updated in
    place.  Returns (x, info) with iterations, relative residual (recursive),
    convergence and breakdown flags (p^T A p <= 0)."""
    r = ops.empty_like(b)
    apply(x, r)
    ops.axpby(1.0, b, -1.0, r)  # r = b - A x
    p = ops.empty_like(b)
    ops.copy(p, r)
    Ap = ops.empty_like(b)
    rr = ops.dot(r, r)
    bnorm = math.sqrt(ops.dot(b, b)) if rnorm0 is None else rnorm0
    info = {"iterations": 0, "converged": False, "breakdown": False, "rel_residual": None}
    if bnorm == 0.0:
        info.update(converged=True, rel_residual=0.0)
        return x, info
    target = (rtol * bnorm) ** 2
    it = 0
    while it < maxiter:
        if rr <= target:
            info["converged"] = True
            break
        apply(p, Ap)
        pAp = ops.dot(p, Ap)
        if not (pAp > 0.0) or not math.isfinite(pAp):
            info["breakdown"] = True
            break
        alpha = rr / pAp
        ops.axpby(alpha, p, 1.0, x)
        ops.axpby(-alpha, Ap, 1.0, r)
        rr_new = ops.dot(r, r)
        beta = rr_new / rr
        ops.axpby(1.0, r, beta, p)
        rr = rr_new
        it += 1
    info["iterations"] = it
    info["rel_residual"] = math.sqrt(max(rr, 0.0)) / bnorm
    if rr <= target:
        info["converged"] = True
    return x, info


def defect_correction(apply64, apply32, b, ops, tol=1e-10, inner_rtol=1e-4, max_outer=60, max_inner=20000,
                      stagnation_factor=0.5, stagnation_window=3):
    """Solve A u = b to ||b - A u|| <= tol ||b|| with the residual b - A u
    and the update u += d in FP64 and the correction A d = r solved by CG in
    FP32 (the residual is scaled to unit norm before the cast).

    Returns (u, info): outer steps, total inner iterations, relative residual
    history (FP64), and a stagnation flag (no reduction by
    `stagnation_factor` over `stagnation_window` outer steps)."""
    u = ops.zeros_like(b)
    r = ops.empty_like(b)
    ops.copy(r, b)
    bnorm = math.sqrt(ops.dot(b, b))
    hist = []
    inner_total = 0
    info = {"outer": 0, "inner_iterations": 0, "converged": False, "stagnated": False, "history": hist,
            "inner_breakdown": False}
    if bnorm == 0.0:
        info["converged"] = True
        return u, info
    r32 = ops.empty_like(b, ops.f32())
    d32 = ops.empty_like(b, ops.f32())
    d64 = ops.empty_like(b)
    for k in range(max_outer + 1):
        rnorm = math.sqrt(ops.dot(r, r))
        hist.append(rnorm / bnorm)
        if rnorm <= tol * bnorm:
            info["converged"] = True
            break
        if len(hist) > stagnation_window and hist[-1] > stagnation_factor * hist[-1 - stagnation_window]:
            info["stagnated"] = True
            break
        if k == max_outer:
            break
        # r32 = r / ||r||
        ops.copy(r32, r)
        ops.axpby(0.0, r32, 1.0 / rnorm, r32)
        d32 = ops.zeros_like(r32)
        _, ii = cg(apply32, r32, d32, ops, rtol=inner_rtol, maxiter=max_inner)
        inner_total += ii["iterations"]
        info["inner_breakdown"] |= ii["breakdown"]
        ops.copy(d64, d32)
        ops.axpby(rnorm, d64, 1.0, u)  # u += ||r|| d
        apply64(u, r)
        ops.axpby(1.0, b, -1.0, r)  # r = b - A u
        info["outer"] = k + 1
    info["inner_iterations"] = inner_total
    info["rel_residual"] = hist[-1]
    return u, info


def device_cg(op, b, x, rtol=1e-10, maxiter=100000, chunk=32, rnorm0=None, progress=None):
    """CG for op's matrix with every iteration on the device
    (`ufem_cg_iterate`): the host reads the residual norm once per `chunk`
    iterations, so up to chunk - 1 iterations beyond the target may run.
    b, x: device tensors of one precision (x updated in place).  progress,
    if given, is called with (iterations, relative residual) after every
    chunk.  Returns (x, info) like `cg`."""
    import torch

    ops = DeviceOps(b.device.index or 0)
    prec = ops._prec(b)
    r = torch.empty_like(b)
    op.apply(x, r)
    ops.axpby(1.0, b, -1.0, r)  # r = b - A x
    p = r.clone()
    ap = torch.empty_like(b)
    scal = torch.zeros(4, dtype=torch.float64, device=b.device)
    L.check(L.lib().ufem_dot(prec, r.numel(), C.c_void_p(r.data_ptr()), C.c_void_p(r.data_ptr()),
                             C.c_void_p(scal.data_ptr()), ops._stream()))
    bnorm = math.sqrt(ops.dot(b, b)) if rnorm0 is None else rnorm0
    info = {"iterations": 0, "converged": False, "breakdown": False, "rel_residual": None}
    if bnorm == 0.0:
        info.update(converged=True, rel_residual=0.0)
        return x, info
    target = (rtol * bnorm) ** 2
    it = 0
    rr = float(scal[0].item())
    while rr > target and it < maxiter:
        n = min(chunk, maxiter - it)
        L.check(L.lib().ufem_cg_iterate(op._h, prec, n, C.c_void_p(x.data_ptr()), C.c_void_p(r.data_ptr()),
                                        C.c_void_p(p.data_ptr()), C.c_void_p(ap.data_ptr()),
                                        C.c_void_p(scal.data_ptr()), ops._stream()))
        it += n
        sc = scal.cpu()
        rr = float(sc[0])
        if progress is not None:
            progress(it, math.sqrt(max(rr, 0.0)) / bnorm)
        if sc[3] != 0.0:
            info["breakdown"] = True
            break
    info["iterations"] = it
    info["rel_residual"] = math.sqrt(max(rr, 0.0)) / bnorm
    info["converged"] = rr <= target
    return x, info


def device_defect_correction(op, b, tol=1e-10, inner_rtol=1e-4, max_outer=60, max_inner=100000, chunk=32,
                             stagnation_factor=0.5, stagnation_window=3, progress=None):
    """`defect_correction` with the FP32 inner solves done by `device_cg`
    (b: float64 device tensor); an inner solve stops at inner_rtol or, when
    less is needed to reach tol, at 0.3 tol ||b|| / ||r|| (at most 1e-2).
    Returns (u, info) like `defect_correction`."""
    import torch

    ops = DeviceOps(b.device.index or 0)
    u = torch.zeros_like(b)
    r = b.clone()
    bnorm = math.sqrt(ops.dot(b, b))
    hist = []
    inner_total = 0
    info = {"outer": 0, "inner_iterations": 0, "converged": False, "stagnated": False, "history": hist,
            "inner_breakdown": False}
    if bnorm == 0.0:
        info["converged"] = True
        return u, info
    r32 = torch.empty(b.numel(), dtype=torch.float32, device=b.device)
    d64 = torch.empty_like(b)
    for k in range(max_outer + 1):
        rnorm = math.sqrt(ops.dot(r, r))
        hist.append(rnorm / bnorm)
        if rnorm <= tol * bnorm:
            info["converged"] = True
            break
        if len(hist) > stagnation_window and hist[-1] > stagnation_factor * hist[-1 - stagnation_window]:
            info["stagnated"] = True
            break
        if k == max_outer:
            break
        ops.copy(r32, r)
        ops.axpby(0.0, r32, 1.0 / rnorm, r32)  # r32 = r / ||r||
        d32 = torch.zeros_like(r32)
        # the last correction only has to close the remaining gap to tol
        rtol_k = min(1e-2, max(inner_rtol, 0.3 * tol * bnorm / rnorm))
        _, ii = device_cg(op, r32, d32, rtol=rtol_k, maxiter=max_inner, chunk=chunk, rnorm0=1.0, progress=progress)
        inner_total += ii["iterations"]
        info["inner_breakdown"] |= ii["breakdown"]
        ops.copy(d64, d32)
        ops.axpby(rnorm, d64, 1.0, u)  # u += ||r|| d
        op.apply(u, r)
        ops.axpby(1.0, b, -1.0, r)  # r = b - A u
        info["outer"] = k + 1
    info["inner_iterations"] = inner_total
    info["rel_residual"] = hist[-1]
    return u, info


def device_reliable_cg(op, b, tol=1e-10, delta=0.1, maxiter=400000, chunk=32, progress=None):
    """CG with its iterations in FP32 on the device (`ufem_cg_iterate`) and
    reliable updates in FP64: the FP32 iterate y is a correction to the FP64
    solution u of A u = b (b: float64 device tensor).  Whenever the FP32
    recursive residual has dropped by `delta` since the last update (or its
    estimate reaches tol ||b||), u += s y in FP64, the true residual
    r = b - A u is formed with the FP64 apply and replaces the FP32 residual
    (scaled to unit norm, s = ||r||), y restarts from zero and the search
    direction p is kept, rescaled to the new unit: unlike a restarted defect
    correction, the FP32 iterations go on in the Krylov space built so far.
    Converged when an update finds ||b - A u|| <= tol ||b|| (FP64).
    Returns (u, info): FP32 iterations, updates, FP64 relative residual."""
    import torch

    ops = DeviceOps(b.device.index or 0)
    stream = ops._stream()
    n = b.numel()
    u = torch.zeros_like(b)
    r = b.clone()
    bnorm = math.sqrt(ops.dot(b, b))
    info = {"iterations": 0, "updates": 0, "converged": False, "breakdown": False, "rel_residual": None}
    if bnorm == 0.0:
        info.update(converged=True, rel_residual=0.0)
        return u, info
    s = bnorm
    r32 = torch.empty(n, dtype=torch.float32, device=b.device)
    ops.copy(r32, r)
    ops.axpby(0.0, r32, 1.0 / s, r32)  # r32 = r / s
    p32 = r32.clone()
    y32 = torch.zeros_like(r32)
    ap32 = torch.empty_like(r32)
    y64 = torch.empty_like(b)
    scal = torch.zeros(4, dtype=torch.float64, device=b.device)

    def set_rr():
        L.check(L.lib().ufem_dot(L.F32, n, C.c_void_p(r32.data_ptr()), C.c_void_p(r32.data_ptr()),
                                 C.c_void_p(scal.data_ptr()), stream))

    set_rr()
    it = 0
    res = 1.0
    while it < maxiter:
        k = min(chunk, maxiter - it)
        L.check(L.lib().ufem_cg_iterate(op._h, L.F32, k, C.c_void_p(y32.data_ptr()), C.c_void_p(r32.data_ptr()),
                                        C.c_void_p(p32.data_ptr()), C.c_void_p(ap32.data_ptr()),
                                        C.c_void_p(scal.data_ptr()), stream))
        it += k
        sc = scal.cpu()
        rr = max(float(sc[0]), 0.0)
        if sc[3] != 0.0:
            info["breakdown"] = True
        if rr > delta * delta and s * math.sqrt(rr) > tol * bnorm and not info["breakdown"] and it < maxiter:
            continue
        # reliable update: u += s y, r = b - A u in FP64
        ops.copy(y64, y32)
        ops.axpby(s, y64, 1.0, u)
        y32.zero_()
        op.apply(u, r)
        ops.axpby(1.0, b, -1.0, r)
        rn = math.sqrt(ops.dot(r, r))
        info["updates"] += 1
        res = rn / bnorm
        if progress is not None:
            progress(it, res)
        if rn <= tol * bnorm or info["breakdown"] or rn == 0.0:
            break
        ops.copy(r32, r)
        ops.axpby(0.0, r32, 1.0 / rn, r32)  # r32 = r / rn
        ops.axpby(0.0, p32, s / rn, p32)    # p in the new unit
        s = rn
        set_rr()
    info["iterations"] = it
    info["rel_residual"] = res
    info["converged"] = res <= tol
    return u, info


def timed(fn, ops):
    ops.sync()
    t0 = time.perf_counter()
    out = fn()
    ops.sync()
    return out, time.perf_counter() - t0
