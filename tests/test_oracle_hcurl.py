"""Pins of the Nedelec oracle (oracle/hcurl.py) against what the mathematics fixes.

* dof counts of the order-p Nedelec space on n1 x n2 x n3 lattices (p per edge,
  2p(p-1) per face, 3p(p-1)^2 per element);
* the reference basis is nodal for its vector dofs: e_a . N_j(node_i) = delta_ij;
* the de Rham property: the ND dofs of the gradient of any H1 function of the same
  order (computed element by element) agree between the elements sharing a dof,
  grad maps into the ND space exactly, so G^T M G equals the H1 stiffness matrix
  (an oracle pinned on its own), and the curl-curl matrix annihilates G;
* on affine meshes the rotation field u = (-y, x, 0) lies in the space: its energy
  is int |curl u|^2 = 4 |Omega| and its mass int (x^2 + y^2) = 2/3 on the unit cube;
* brute force on tiny meshes: the unconstrained curl-curl matrix has a null space of
  exactly the dimension of the gradients (H1 dofs - 1) and the mass matrix is SPD.
A wrong sign or permutation of shared dofs, a transposed Jacobian in either map or a
dropped curl term breaks at least one of these.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import forms, hcurl


def _counts(n, p):
    nx, ny, nz = n
    edges = nx * (ny + 1) * (nz + 1) + ny * (nx + 1) * (nz + 1) + nz * (nx + 1) * (ny + 1)
    faces = nx * ny * (nz + 1) + ny * nz * (nx + 1) + nx * nz * (ny + 1)
    return edges * p + faces * 2 * p * (p - 1) + nx * ny * nz * 3 * p * (p - 1) ** 2


@pytest.mark.parametrize("n,p", [((1, 1, 1), 1), ((2, 2, 2), 1), ((2, 3, 2), 2),
                                 ((3, 2, 2), 3), ((2, 1, 1), 5)])
def test_dof_counts(n, p):
    S = hcurl.NDSpace(synth.hex_lattice(n, 0.1, seed=1, rotate_seed=3), p)
    assert S.ndofs == _counts(n, p)
    # boundary dofs of one element: all of them except the 3p(p-1)^2 interior ones
    if n == (1, 1, 1):
        assert S.boundary.sum() == S.ndofs - 3 * p * (p - 1) ** 2


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_reference_basis_is_nodal(p):
    pts, axis = hcurl.nd_node_points(p)
    N, _ = hcurl.nd_reference_basis(p, pts)                       # [node, basis, 3]
    vals = N[np.arange(len(axis)), :, axis]                       # e_{a_i} . N_j(node_i)
    assert np.abs(vals - np.eye(len(axis))).max() < 1e-12


def _gradient_setup(mesh, p):
    S = hcurl.NDSpace(mesh, p)
    H = oracle.H1Space(mesh, p)
    G, spread = hcurl.discrete_gradient(S, H)
    return S, H, G, spread


@pytest.mark.parametrize("p", [1, 2, 3])
def test_gradient_maps_exactly_into_nd(p):
    mesh = synth.hex_lattice((2, 2, 1), 0.15, seed=4, rotate_seed=9)
    S, H, G, spread = _gradient_setup(mesh, p)
    assert spread < 1e-12                      # orientation of shared dofs is consistent
    q = p + 2
    M = hcurl.assemble_nd(S, hcurl.element_nd_mass(mesh, p, q))
    K = oracle.assemble(H, forms.element_stiffness(mesh, p, q))
    GtMG = (G.T @ M @ G).toarray()
    Kd = K.toarray()
    assert np.abs(GtMG - Kd).max() < 1e-12 * np.abs(Kd).max()
    C = hcurl.assemble_nd(S, hcurl.element_nd_curlcurl(mesh, p, q))
    CG = (C @ G).toarray()
    assert np.abs(CG).max() < 1e-12 * np.abs(C.toarray()).max()


def test_gradient_pin_catches_a_flipped_sign():
    """Mutation: flipping the sign of one shared dof in one element breaks the pin."""
    mesh = synth.hex_lattice((2, 1, 1), 0.1, seed=2)
    S, H, G, spread = _gradient_setup(mesh, 2)
    assert spread < 1e-12
    shared = np.intersect1d(S.elem_dofs[0], S.elem_dofs[1])
    j = int(np.nonzero(S.elem_dofs[1] == shared[0])[0][0])
    S.elem_signs[1, j] *= -1.0
    _, spread2 = hcurl.discrete_gradient(S, H)
    assert spread2 > 1e-3


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rotation_field_energy_on_affine_mesh(p):
    mesh = synth.hex_lattice((3, 2, 2), 0.0, seed=0, rotate_seed=5)
    S = hcurl.NDSpace(mesh, p)
    u = hcurl.nd_interpolate(S, lambda x: np.stack([-x[..., 1], x[..., 0], 0 * x[..., 2]], axis=-1))
    q = p + 2
    C = hcurl.assemble_nd(S, hcurl.element_nd_curlcurl(mesh, p, q))
    M = hcurl.assemble_nd(S, hcurl.element_nd_mass(mesh, p, q))
    assert abs(u @ (C @ u) - 4.0) < 1e-12
    assert abs(u @ (M @ u) - 2.0 / 3.0) < 1e-12


@pytest.mark.parametrize("p", [2, 3])
def test_linear_field_energy_on_affine_mesh(p):
    """From p = 2 every linear field is in the space: u = A x with A general."""
    A = np.array([[0.3, -1.0, 0.2], [0.7, 0.1, -0.4], [0.5, 0.9, -0.2]])
    mesh = synth.hex_lattice((2, 2, 2), 0.0, seed=0, rotate_seed=7)
    S = hcurl.NDSpace(mesh, p)
    u = hcurl.nd_interpolate(S, lambda x: x @ A.T)
    q = p + 2
    C = hcurl.assemble_nd(S, hcurl.element_nd_curlcurl(mesh, p, q))
    M = hcurl.assemble_nd(S, hcurl.element_nd_mass(mesh, p, q))
    curl = np.array([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    assert abs(u @ (C @ u) - curl @ curl) < 1e-12
    # int_{[0,1]^3} (A x).(A x) = sum_ab (A^T A)_ab int x_a x_b; int x_a x_b = 1/4 (a != b), 1/3
    AtA = A.T @ A
    want = np.trace(AtA) / 3.0 + (AtA.sum() - np.trace(AtA)) / 4.0
    assert abs(u @ (M @ u) - want) < 1e-12


@pytest.mark.parametrize("n,p", [((2, 1, 1), 1), ((2, 2, 1), 1), ((2, 1, 1), 2)])
def test_curlcurl_null_space_dimension(n, p):
    mesh = synth.hex_lattice(n, 0.15, seed=6, rotate_seed=2)
    S = hcurl.NDSpace(mesh, p)
    H = oracle.H1Space(mesh, p)
    q = p + 2
    C = hcurl.assemble_nd(S, hcurl.element_nd_curlcurl(mesh, p, q)).toarray()
    M = hcurl.assemble_nd(S, hcurl.element_nd_mass(mesh, p, q)).toarray()
    assert np.abs(C - C.T).max() < 1e-13 and np.abs(M - M.T).max() < 1e-13
    ev = np.linalg.eigvalsh(C)
    nullity = int((np.abs(ev) < 1e-10 * np.abs(ev).max()).sum())
    assert nullity == H.ndofs - 1
    assert np.linalg.eigvalsh(M).min() > 0.0
