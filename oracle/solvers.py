"""Preconditioned CG and L2 error (oracle; test infrastructure only).

* CG on the assembled, constrained operator -- "Scalable Linear Solvers" (the
  ex1p listing: CGSolver with SetRelTol / SetMaxIter, unpreconditioned in
  partial assembly).  The Jacobi (diagonal) preconditioner is an addition.
  Stopping test (the paper does not define the norm of SetRelTol): the
  recursive residual ||r_k||_2 / ||b||_2 <= tol, x_0 = 0; the true residual
  is recomputed at exit and reported.
* L2 error ||u_h - u||_{L2} by quadrature with p+4 points per direction
  (GridFunction::ComputeL2Error in "Discrete de Rham Complex").

Pins: CG agrees with scipy's sparse direct solve; the A-norm of the error
decreases monotonically; L2 rates (tests/test_oracle_solvers.py).
"""
import numpy as np

from .basis import tensor_basis
from .forms import quadrature_points
from .geometry import map_points
from .quadrature import gauss_lobatto


def pcg(A, b, diag=None, tol=1e-10, maxiter=2000, x0=None):
    """Textbook PCG with M = diag(diag) (None means no preconditioner).

    Returns dict(x, iters, converged, history, true_rel_res) where history holds
    ||r_k|| / ||b|| for k = 0..iters.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return {"x": x, "iters": 0, "converged": True, "history": [0.0], "true_rel_res": 0.0}
    minv = None if diag is None else 1.0 / np.asarray(diag, dtype=np.float64)
    z = r if minv is None else minv * r
    d = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r) / bnorm]
    converged = hist[0] <= tol
    k = 0
    while not converged and k < maxiter:
        q = A @ d
        dq = d @ q
        if not dq > 0.0:
            break
        alpha = rz / dq
        x += alpha * d
        r -= alpha * q
        k += 1
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= tol:
            converged = True
            break
        z = r if minv is None else minv * r
        rz_new = r @ z
        d = z + (rz_new / rz) * d
        rz = rz_new
    true_rel = np.linalg.norm(b - A @ x) / bnorm
    return {"x": x, "iters": k, "converged": converged, "history": hist,
            "true_rel_res": true_rel}


def l2_error(space, u_dofs, u_exact, extra=4):
    """||u_h - u_exact||_{L2(Omega)} with (p + extra)^3 Gauss points per element."""
    q1d = space.p + extra
    pts, w = quadrature_points(q1d)
    x, J = map_points(space.mesh, pts)
    det = np.linalg.det(J)
    val, _ = tensor_basis(gauss_lobatto(space.p + 1), pts)
    uh = np.einsum("qi,ei->eq", val, np.asarray(u_dofs)[space.elem_dofs])
    err = (uh - u_exact(x)) ** 2
    return float(np.sqrt(np.sum(err * det * w[None, :])))
