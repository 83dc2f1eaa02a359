"""Pins for the oracle's H1 space (dof identification, numbering, boundary) -- CPU only."""
import numpy as np
import pytest

import oracle
import synth
from oracle import forms


@pytest.mark.parametrize("n,p", [(1, 1), (2, 3), (3, 2), (3, 4)])
def test_counts(n, p):
    s = oracle.H1Space(synth.hex_lattice(n, 0.1, seed=n), p)
    m = n * p + 1
    assert s.ndofs == m ** 3
    assert s.boundary.sum() == m ** 3 - max(m - 2, 0) ** 3
    # numbering order: all vertex dofs, then edge, face and interior dofs
    assert np.all(np.diff(s.dof_class) >= 0)
    assert set(np.unique(s.dof_class)) <= {1, 2, 4, 8}


def test_boundary_dofs_are_on_the_cube_surface():
    s = oracle.H1Space(synth.hex_lattice(4, 0.1, seed=3), 3)
    X = s.dof_coordinates()
    on_surface = np.any((np.abs(X) < 1e-12) | (np.abs(X - 1) < 1e-12), axis=1)
    assert np.array_equal(on_surface, s.boundary)


def test_shared_nodes_consistent():
    mesh = synth.hex_lattice(3, 0.1, seed=5, rotate_seed=8)
    s = oracle.H1Space(mesh, 3)
    from oracle.basis import tensor_points
    from oracle.quadrature import gauss_lobatto
    x, _ = oracle.map_points(mesh, tensor_points(gauss_lobatto(4)))
    X = s.dof_coordinates()
    np.testing.assert_allclose(x.reshape(-1, 3), X[s.elem_dofs.ravel()], atol=1e-14)


def _match(Xa, Xb):
    ka = np.lexsort(np.round(Xa, 9).T[::-1])
    kb = np.lexsort(np.round(Xb, 9).T[::-1])
    perm = np.empty(len(Xa), dtype=np.int64)
    perm[ka] = kb
    assert np.allclose(Xa, Xb[perm], atol=1e-12)
    return perm


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rotation_invariance(p):
    """Relabelling every element's vertices by a random rotation leaves the operator unchanged."""
    base = synth.hex_lattice(3, 0.1, seed=12)
    rot = synth.hex_lattice(3, 0.1, seed=12, rotate_seed=99)
    assert not np.array_equal(base["hex"], rot["hex"])
    sa, sb = oracle.H1Space(base, p), oracle.H1Space(rot, p)
    Ka = oracle.assemble(sa, forms.element_stiffness(base, p, p + 2)).toarray()
    Kb = oracle.assemble(sb, forms.element_stiffness(rot, p, p + 2)).toarray()
    perm = _match(sa.dof_coordinates(), sb.dof_coordinates())
    np.testing.assert_allclose(Ka, Kb[np.ix_(perm, perm)], atol=1e-12)
    assert np.array_equal(sa.boundary, sb.boundary[perm])
