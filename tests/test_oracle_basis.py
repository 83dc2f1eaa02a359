"""Pins for the oracle's quadrature and basis (CPU only).

Each check is against mathematics fixed independently of the oracle's code:
monomial integrals, closed-form Gauss-Lobatto nodes, the nodal (Kronecker delta)
property of Lagrange bases, and exact reproduction of polynomials.
"""
import json
import os

import numpy as np
import pytest

from oracle.basis import lagrange_derivatives, lagrange_values, tensor_basis, tensor_points
from oracle.quadrature import gauss_legendre, gauss_lobatto, gauss_lobatto_weights

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("q", range(1, 11))
def test_gauss_exact_on_monomials(q):
    x, w = gauss_legendre(q)
    assert abs(w.sum() - 1.0) < 1e-14
    for k in range(2 * q):
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 1e-14
    # degree 2q is not integrated exactly: the rule really has q points
    assert abs(np.dot(w, x ** (2 * q)) - 1.0 / (2 * q + 1)) > 1e-13


def test_lobatto_closed_forms():
    with open(os.path.join(GOLDEN, "gauss_lobatto_closed_forms.json")) as fh:
        table = json.load(fh)["nodes_on_unit_interval"]
    for p, expr in table.items():
        expected = np.array([eval(e, {"sqrt": np.sqrt}) for e in expr])
        np.testing.assert_allclose(gauss_lobatto(int(p) + 1), expected, atol=1e-15)


@pytest.mark.parametrize("p", range(1, 9))
def test_lobatto_rule_exactness(p):
    x, w = gauss_lobatto(p + 1), gauss_lobatto_weights(p + 1)
    assert x[0] == 0.0 and x[-1] == 1.0 and np.all(np.diff(x) > 0)
    for k in range(2 * p):
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 1e-13


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_nodal_and_reproduction(p):
    nodes = gauss_lobatto(p + 1)
    np.testing.assert_allclose(lagrange_values(nodes, nodes), np.eye(p + 1), atol=1e-13)
    xs = np.linspace(0.0, 1.0, 37)
    L, dL = lagrange_values(nodes, xs), lagrange_derivatives(nodes, xs)
    np.testing.assert_allclose(L.sum(axis=1), 1.0, atol=1e-12)
    np.testing.assert_allclose(dL.sum(axis=1), 0.0, atol=1e-10)
    rng = np.random.default_rng(p)
    c = rng.normal(size=p + 1)                      # random polynomial of degree p
    poly = np.polynomial.Polynomial(c)
    np.testing.assert_allclose(L @ poly(nodes), poly(xs), atol=1e-11)
    np.testing.assert_allclose(dL @ poly(nodes), poly.deriv()(xs), atol=1e-9)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_tensor_basis_gradient_and_reproduction(p):
    nodes = gauss_lobatto(p + 1)
    rng = np.random.default_rng(10 + p)
    pts = rng.uniform(size=(11, 3))
    val, grad = tensor_basis(nodes, pts)
    # gradients against central differences of the values
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        vp, _ = tensor_basis(nodes, pts + e)
        vm, _ = tensor_basis(nodes, pts - e)
        np.testing.assert_allclose(grad[a], (vp - vm) / (2 * h), atol=1e-6)
    # a product of 1D polynomials of degree p lies in Q_p and is reproduced
    cs = [np.polynomial.Polynomial(rng.normal(size=p + 1)) for _ in range(3)]
    f = lambda X: cs[0](X[:, 0]) * cs[1](X[:, 1]) * cs[2](X[:, 2])
    nodal = f(tensor_points(nodes))
    np.testing.assert_allclose(val @ nodal, f(pts), atol=1e-10)
    # lexicographic order: dof 1 is the second node along the first axis
    assert np.allclose(tensor_points(nodes)[1], [nodes[1], 0.0, 0.0])
