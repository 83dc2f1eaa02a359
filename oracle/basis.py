"""Nodal Lagrange bases (oracle; test infrastructure only).

The H1 basis of order p is the nodal Lagrange basis at the p+1 Gauss-Lobatto
points ("Finite Elements": nodal elements satisfy phi_j(node_i) = delta_ij).  On
the hexahedron the basis is the tensor product of 1D bases; here the 3D values
and gradients are evaluated *directly* at 3D points as products of 1D Lagrange
polynomials, and stored as dense [npts, ndof] matrices -- the matrix B with
B_ki = phi_i(xhat_k) of "High-Order Partial Assembly", never factorised.

Local dof order: lexicographic, i = i1 + D1*(i2 + D1*i3), i1 along xhat_1.

Pins: delta property, partition of unity, derivative sums vanish, exact
interpolation of polynomials of degree <= p (tests/test_oracle_basis.py).
"""
import numpy as np


def lagrange_values(nodes, x):
    """L[k, j] = prod_{m != j} (x_k - n_m) / (n_j - n_m)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    out = np.ones((x.size, n))
    for j in range(n):
        for m in range(n):
            if m != j:
                out[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return out


def lagrange_derivatives(nodes, x):
    """dL[k, j] = d/dx of the j-th Lagrange polynomial at x_k (product rule)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    out = np.zeros((x.size, n))
    for j in range(n):
        for l in range(n):
            if l == j:
                continue
            term = np.full(x.size, 1.0 / (nodes[j] - nodes[l]))
            for m in range(n):
                if m != j and m != l:
                    term *= (x - nodes[m]) / (nodes[j] - nodes[m])
            out[:, j] += term
    return out


def tensor_basis(nodes, points):
    """Values [npts, D^3] and reference gradients [3, npts, D^3] of the 3D basis.

    ``points`` is [npts, 3]; dof i = (i1, i2, i3) lexicographic with i1 fastest.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.asarray(points, dtype=np.float64)
    d1 = nodes.size
    v = [lagrange_values(nodes, pts[:, a]) for a in range(3)]       # [npts, D1]
    g = [lagrange_derivatives(nodes, pts[:, a]) for a in range(3)]
    i3, i2, i1 = np.meshgrid(np.arange(d1), np.arange(d1), np.arange(d1), indexing="ij")
    i1, i2, i3 = i1.ravel(), i2.ravel(), i3.ravel()
    val = v[0][:, i1] * v[1][:, i2] * v[2][:, i3]
    grad = np.stack([g[0][:, i1] * v[1][:, i2] * v[2][:, i3],
                     v[0][:, i1] * g[1][:, i2] * v[2][:, i3],
                     v[0][:, i1] * v[1][:, i2] * g[2][:, i3]])
    return val, grad


def tensor_points(x1d):
    """3D tensor points [n^3, 3] with the first coordinate fastest."""
    x1d = np.asarray(x1d, dtype=np.float64)
    z, y, x = np.meshgrid(x1d, x1d, x1d, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def tensor_weights(w1d):
    """Tensor weights [n^3] in the same order as :func:`tensor_points`."""
    w1d = np.asarray(w1d, dtype=np.float64)
    z, y, x = np.meshgrid(w1d, w1d, w1d, indexing="ij")
    return (x * y * z).ravel()
