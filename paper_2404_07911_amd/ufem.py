"""Python face of libufem: plans, device operators and the autograd wrapper.

Only argument marshalling lives here; every step of the operator runs in the
HIP kernels of libufem.so.  Torch provides device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np

from . import _lib as L


@dataclasses.dataclass
class Problem:
    """Unfitted SIPG Poisson problem on [lo, hi]^dim cut by a union of balls,
    or with ``plane = (normal, offset)`` by the half space n . x < offset
    (Sections 2.1-2.2 of the paper; face ghost penalty on cut-cell faces)."""

    dim: int
    n: int
    degree: int
    centers: np.ndarray
    radii: np.ndarray
    lo: float = -1.0
    hi: float = 1.0
    q_cut: int = 0
    max_depth: int = 4
    nitsche_factor: float = 20.0
    sipg_factor: float = 20.0
    gp_gamma: float = 0.1
    gp_jmin: int = 0
    gp_flat: bool = False
    plane: tuple | None = None
    gp_kind: str = "face"  # "face", "volume" (stable neighbours) or "volume_all"
    space: str = "dg"  # "dg" (SIPG) or "cg" (continuous FE_Q)

    @classmethod
    def from_workload(cls, wl, **kw):
        kw.setdefault("plane", getattr(wl, "plane", None))
        return cls(wl.dim, wl.n, wl.degree, np.asarray(wl.centers), np.asarray(wl.radii), wl.lo, wl.hi, **kw)

    def _struct(self):
        c = np.ascontiguousarray(np.asarray(self.centers, dtype=np.float64).reshape(-1, self.dim))
        r = np.ascontiguousarray(np.asarray(self.radii, dtype=np.float64).reshape(-1))
        s = L.ufem_problem()
        s.dim = self.dim
        s.n = self.n
        s.lo = self.lo
        s.hi = self.hi
        s.degree = self.degree
        s.q_cut = self.q_cut
        s.max_depth = self.max_depth
        s.n_balls = r.size
        s.centers = c.ctypes.data_as(C.POINTER(C.c_double))
        s.radii = r.ctypes.data_as(C.POINTER(C.c_double))
        s.nitsche_factor = self.nitsche_factor
        s.sipg_factor = self.sipg_factor
        s.gp_gamma = self.gp_gamma
        s.gp_jmin = self.gp_jmin
        s.gp_flat = int(bool(self.gp_flat))
        kinds = {"face": L.GP_FACE, "volume": L.GP_VOLUME, "volume_all": L.GP_VOLUME_ALL}
        if self.gp_kind not in kinds:
            raise ValueError(f"gp_kind must be one of {sorted(kinds)}")
        s.gp_kind = kinds[self.gp_kind]
        if self.space not in ("dg", "cg"):
            raise ValueError("space must be 'dg' or 'cg'")
        s.space = L.SPACE_CG if self.space == "cg" else L.SPACE_DG
        if self.plane is not None:
            nrm = np.asarray(self.plane[0], dtype=np.float64).reshape(-1)
            s.levelset = L.LEVELSET_PLANE
            for a in range(min(3, nrm.size)):
                s.plane_normal[a] = float(nrm[a])
            s.plane_offset = float(self.plane[1])
        return s, (c, r)


class Plan:
    """Host plan (classification, faces, cut quadrature, layouts).  No GPU."""

    def __init__(self, problem: Problem):
        self.problem = problem
        s, keep = problem._struct()
        h = C.c_void_p()
        L.check(L.lib().ufem_plan_create(C.byref(s), C.byref(h)))
        self._h = h
        del keep
        inf = L.ufem_info()
        L.check(L.lib().ufem_plan_info(self._h, C.byref(inf)))
        self.info = inf.as_dict()

    def __del__(self):
        h = getattr(self, "_h", None)
        try:
            if h is not None and h.value:
                L.lib().ufem_plan_destroy(h)
        except Exception:  # interpreter shutdown
            pass
        self._h = None

    @property
    def handle(self):
        return self._h

    def cells(self) -> np.ndarray:
        out = np.zeros(self.info["n_background"], dtype=np.int8)
        L.check(L.lib().ufem_plan_cells(self._h, out.ctypes.data))
        return out

    def faces(self) -> np.ndarray:
        out = np.zeros((self.info["n_faces"], 5), dtype=np.int32)
        if out.size:
            L.check(L.lib().ufem_plan_faces(self._h, out.ctypes.data))
        return out

    def import_quadrature(self, vol_count, face_count, surf_count, ref, w, nrm):
        """Replace the cut rules (layout of ufem_plan_import_quadrature: point
        counts per cut cell / cut face / cut cell, then reference points,
        weights and normals of the three segments in kappa order)."""
        d = self.problem.dim
        vc = np.ascontiguousarray(vol_count, dtype=np.int64)
        fc = np.ascontiguousarray(face_count, dtype=np.int64)
        sc = np.ascontiguousarray(surf_count, dtype=np.int64)
        if vc.size != self.info["n_cut"] or sc.size != self.info["n_cut"] or fc.size != self.info["n_faces_cut"]:
            raise ValueError("one count per cut cell, cut face and cut cell")
        n = int(vc.sum() + fc.sum() + sc.sum())
        r = np.ascontiguousarray(ref, dtype=np.float64).reshape(-1)
        wt = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
        nm = np.ascontiguousarray(nrm, dtype=np.float64).reshape(-1)
        if r.size != n * d or wt.size != n or nm.size != n * d:
            raise ValueError(f"expected {n} points ({n * d} coordinates)")
        L.check(L.lib().ufem_plan_import_quadrature(self._h, vc.ctypes.data, fc.ctypes.data, sc.ctypes.data,
                                                    r.ctypes.data, wt.ctypes.data, nm.ctypes.data))
        inf = L.ufem_info()
        L.check(L.lib().ufem_plan_info(self._h, C.byref(inf)))
        self.info = inf.as_dict()

    def qp(self):
        """Physical points, reference points, reference weights, normals of
        every quadrature point in kappa order."""
        n, d = self.info["n_qp"], self.problem.dim
        xyz = np.zeros((n, d))
        ref = np.zeros((n, d))
        w = np.zeros(n)
        nrm = np.zeros((n, d))
        L.check(L.lib().ufem_plan_qp(self._h, xyz.ctypes.data, ref.ctypes.data, w.ctypes.data, nrm.ctypes.data))
        return xyz, ref, w, nrm


def _torch():
    import torch

    return torch


def _prec_of(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return L.F64
    if t.dtype == torch.float32:
        return L.F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Operator:
    """Device operator v = A u on one GPU."""

    def __init__(self, plan: Plan, device: int = 0, max_device_bytes: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("Operator needs a GPU (HIP device); none is available")
        self.plan = plan
        self.device = device
        self.info = dict(plan.info)
        h = C.c_void_p()
        with torch.cuda.device(device):
            L.check(L.lib().ufem_setup(plan.handle, device, None, max_device_bytes, C.byref(h)))
        self._h = h
        self.n_dofs = self.info["n_dofs"]
        self.n_qp = self.info["n_qp"]
        self._kappa = {L.F64: None, L.F32: None}
        self._kappa_src = None
        self.terms = L.TERM_ALL

    def __del__(self):
        h = getattr(self, "_h", None)
        try:
            if h is not None and h.value:
                L.lib().ufem_destroy(h)
        except Exception:  # interpreter shutdown
            pass
        self._h = None

    def _check_vec(self, t, n, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.numel() != n or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with {n} entries, got {tuple(t.shape)}")
        if t.device.index != self.device:
            raise ValueError(f"{name} is on device {t.device}, operator on {self.device}")

    def set_terms(self, mask: int):
        L.check(L.lib().ufem_set_terms(self._h, int(mask)))
        self.terms = int(mask)

    def set_mixed(self, enable: bool, stream=None):
        """Precomputed element matrices for the cut cells' volume and
        interface terms (True) or fully matrix-free evaluation (False)."""
        L.check(L.lib().ufem_set_mixed(self._h, int(bool(enable)), _stream_handle(stream)))

    def set_max_blocks(self, max_blocks: int):
        """Cap the workgroups of every launch (0: sized by the work)."""
        L.check(L.lib().ufem_set_max_blocks(self._h, int(max_blocks)))

    def set_kappa(self, kappa, stream=None):
        """kappa: device tensor of n_qp entries (float64 and/or float32) or None."""
        if kappa is None:
            for p in (L.F64, L.F32):
                L.check(L.lib().ufem_set_kappa(self._h, p, None, None))
                self._kappa[p] = None
            self._kappa_src = None
            return
        torch = _torch()
        self._check_vec(kappa, self.n_qp, "kappa")
        k64 = kappa.to(torch.float64).contiguous()
        k32 = kappa.to(torch.float32).contiguous()
        s = _stream_handle(stream)
        L.check(L.lib().ufem_set_kappa(self._h, L.F64, C.c_void_p(k64.data_ptr()), s))
        L.check(L.lib().ufem_set_kappa(self._h, L.F32, C.c_void_p(k32.data_ptr()), s))
        self._kappa = {L.F64: k64, L.F32: k32}
        self._kappa_src = kappa

    def apply(self, u, v=None, stream=None):
        torch = _torch()
        self._check_vec(u, self.n_dofs, "u")
        if v is None:
            v = torch.empty_like(u)
        self._check_vec(v, self.n_dofs, "v")
        if v.dtype != u.dtype:
            raise TypeError("u and v must share a dtype")
        L.check(L.lib().ufem_apply(self._h, _prec_of(u), C.c_void_p(u.data_ptr()), C.c_void_p(v.data_ptr()),
                                   _stream_handle(stream)))
        return v

    def apply_part(self, part, u, v, stream=None):
        """Kernel stages of the apply (mask of PART_* bits: 1 inside cells,
        2 cut cells' structured faces, 4 cut volume/interface lines, 8 cut-face
        lines; 4 and 8 add to v)."""
        self._check_vec(u, self.n_dofs, "u")
        self._check_vec(v, self.n_dofs, "v")
        if v.dtype != u.dtype:
            raise TypeError("u and v must share a dtype")
        L.check(L.lib().ufem_apply_part(self._h, _prec_of(u), int(part), C.c_void_p(u.data_ptr()),
                                        C.c_void_p(v.data_ptr()), _stream_handle(stream)))
        return v

    def apply_adjoint(self, w, u, atw=None, dkappa=None, want_dkappa=True, stream=None):
        torch = _torch()
        self._check_vec(w, self.n_dofs, "w")
        self._check_vec(u, self.n_dofs, "u")
        if w.dtype != u.dtype:
            raise TypeError("w and u must share a dtype")
        if atw is None:
            atw = torch.empty_like(w)
        self._check_vec(atw, self.n_dofs, "atw")
        if atw.dtype != w.dtype:
            raise TypeError("atw must have the dtype of w")
        if want_dkappa and dkappa is None:
            dkappa = torch.empty(self.n_qp, dtype=w.dtype, device=w.device)
        dk_ptr = C.c_void_p(dkappa.data_ptr()) if dkappa is not None else None
        if dkappa is not None:
            self._check_vec(dkappa, self.n_qp, "dkappa")
            if dkappa.dtype != w.dtype:
                raise TypeError("dkappa must have the dtype of w")
        L.check(L.lib().ufem_apply_adjoint(self._h, _prec_of(w), C.c_void_p(w.data_ptr()),
                                           C.c_void_p(u.data_ptr()), C.c_void_p(atw.data_ptr()), dk_ptr,
                                           _stream_handle(stream)))
        return atw, dkappa


def _make_apply_fn():
    torch = _torch()

    class UfemApply(torch.autograd.Function):
        """v = A(kappa) u with the hand-written adjoint as backward:
        dL/du = A^T dL/dv and dL/dkappa_q = a_q(dL/dv, u)."""

        @staticmethod
        def forward(ctx, u, kappa, op):
            kap = kappa.detach().contiguous() if kappa is not None else None
            op.set_kappa(kap)
            u_in = u.detach().contiguous()
            v = op.apply(u_in)
            # the operator holds one coefficient and one term mask: backward
            # restores the ones of this forward
            ctx.op = op
            ctx.terms = op.terms
            ctx.has_kappa = kap is not None
            ctx.save_for_backward(u_in, kap if kap is not None else u_in.new_empty(0))
            return v

        @staticmethod
        def backward(ctx, grad_v):
            u, kap = ctx.saved_tensors
            op = ctx.op
            prev_kappa, prev_terms = op._kappa_src, op.terms
            op.set_kappa(kap if ctx.has_kappa else None)
            op.set_terms(ctx.terms)
            try:
                atw, dk = op.apply_adjoint(grad_v.contiguous(), u, want_dkappa=ctx.has_kappa)
            finally:
                op.set_kappa(prev_kappa)
                op.set_terms(prev_terms)
            return atw, (dk if ctx.has_kappa else None), None

    return UfemApply


_APPLY_FN = None


def ufem_apply(u, kappa, op):
    """Differentiable v = A(kappa) u (kappa may be None for kappa = 1)."""
    global _APPLY_FN
    if _APPLY_FN is None:
        _APPLY_FN = _make_apply_fn()
    return _APPLY_FN.apply(u, kappa, op)
