"""CPU tests of the solver drivers (CG, mixed-precision defect correction)
with the oracle as the operator: convergence to 1e-10, the FP32 inner
solve, breakdown and stagnation flags."""
import numpy as np
import pytest

import ufem_inputs as ui
from oracle.operator import UnfittedDG
from paper_2404_07911_amd.solvers import HostOps, cg, defect_correction


@pytest.fixture(scope="module")
def problem():
    wl, rng = ui.disk2d(3, n=10, degree=1)
    op = UnfittedDG(wl.dim, wl.n, wl.degree, wl.centers, wl.radii)
    A = op.assemble()
    ustar = ui.uniform_vector(rng, op.n_dofs)
    b = A @ ustar
    return op, A, ustar, b


def _apply(A):
    def f(x, out):
        out[:] = (A @ x.astype(np.float64)).astype(out.dtype)

    return f


def _apply32(A):
    A32 = A.astype(np.float32)

    def f(x, out):
        out[:] = (A32 @ x.astype(np.float32)).astype(np.float32)

    return f


def test_cg_converges_to_1e10(problem):
    op, A, ustar, b = problem
    ops = HostOps()
    x = np.zeros_like(b)
    x, info = cg(_apply(A), b, x, ops, rtol=1e-10, maxiter=5000)
    assert info["converged"] and not info["breakdown"]
    assert np.linalg.norm(b - A @ x) <= 1.5e-10 * np.linalg.norm(b)


def test_defect_correction_fp32_inner(problem):
    op, A, ustar, b = problem
    ops = HostOps()
    u, info = defect_correction(_apply(A), _apply32(A), b, ops, tol=1e-10, inner_rtol=1e-3)
    assert info["converged"] and not info["stagnated"]
    assert info["outer"] >= 2  # FP32 alone cannot reach 1e-10
    assert np.linalg.norm(b - A @ u) <= 1e-10 * np.linalg.norm(b)
    assert info["history"][-1] <= 1e-10


def test_cg_reports_breakdown_on_indefinite_operator(problem):
    op, A, ustar, b = problem
    x = np.zeros_like(b)
    _, info = cg(_apply(-A), b, x, HostOps(), rtol=1e-10, maxiter=50)
    assert info["breakdown"] and not info["converged"]


def test_defect_correction_reports_stagnation(problem):
    op, A, ustar, b = problem
    # an inner operator that is twice the true one: every correction
    # overshoots and the outer residual stops decreasing
    u, info = defect_correction(_apply(A), _apply32(0.5 * A), b, HostOps(), tol=1e-10, inner_rtol=1e-6, max_outer=20)
    assert info["stagnated"] and not info["converged"]
