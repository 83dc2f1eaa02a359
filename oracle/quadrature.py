"""1D quadrature and node sets on [0, 1] (oracle; test infrastructure only).

* Gauss-Legendre points/weights: the quadrature rule {xhat_k, alpha_k} of the
  "High-Order Partial Assembly" section (mass-matrix equations), tensorised.
* Gauss-Lobatto points: the nodes of the nodal Lagrange H1 basis named in
  "Finite Elements" (basis types).

Pins: Gauss exactness for monomials up to degree 2q-1; Lobatto closed forms for
p <= 4 and Lobatto exactness up to degree 2p-1 (tests/test_oracle_basis.py).
"""
import numpy as np
from numpy.polynomial import legendre as _leg


def gauss_legendre(q: int):
    """q-point Gauss-Legendre rule mapped from [-1, 1] to [0, 1]."""
    x, w = _leg.leggauss(int(q))
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto(npts: int):
    """npts Gauss-Lobatto points on [0, 1]: the ends and the roots of P'_{npts-1}."""
    p = int(npts) - 1
    if p < 1:
        raise ValueError("need at least two Lobatto points")
    inner = np.sort(np.real(_leg.Legendre.basis(p).deriv().roots())) if p > 1 else np.array([])
    x = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (x + 1.0)


def gauss_lobatto_weights(npts: int):
    """Lobatto weights on [0, 1]: 2 / (p (p+1) P_p(x)^2) on [-1, 1], halved."""
    p = int(npts) - 1
    x = 2.0 * gauss_lobatto(npts) - 1.0
    pp = _leg.Legendre.basis(p)(x)
    return 0.5 * 2.0 / (p * (p + 1) * pp ** 2)
