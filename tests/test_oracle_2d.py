"""Pins for the 2D (quadrilateral) oracle (CPU only).

Expected values come from outside the oracle: exact 1D integrals of Lagrange
polynomials (Vandermonde solve, symbolic integration) tensorised with Kronecker
products, affine changes of variables, K 1 = 0 and the area, the linear patch test,
the L2 convergence rate, and invariance under relabelled element vertices.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import twod
from tests._common import match_by_coords
from tests.test_oracle_forms import _exact_1d


def _kron2(tx, ty):
    # lexicographic dof index i1 + D*i2: the first axis varies fastest
    return np.kron(ty, tx)


def _single(A=None):
    v = synth.QUAD_CORNERS.astype(np.float64)
    if A is not None:
        v = v @ np.asarray(A).T
    return {"vertices": v, "quad": np.arange(4)[None, :]}


def _matrices(mesh, p, coeff=None):
    S = twod.H1Space2D(mesh, p)
    K = oracle.assemble(S, twod.element_stiffness_2d(mesh, p, p + 2, coeff))
    M = oracle.assemble(S, twod.element_mass_2d(mesh, p, p + 2))
    return S, K, M


@pytest.mark.parametrize("n,p", [(3, 1), (3, 2), (2, 4), (1, 8)])
def test_counts(n, p):
    S = twod.H1Space2D(synth.quad_lattice(n, 0.1, seed=1, rotate_seed=2), p)
    assert S.ndofs == (n * p + 1) ** 2
    assert S.boundary.sum() == 4 * n * p


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_unit_square_element_matrices_exact(p):
    M1, K1, _ = _exact_1d(p)
    mesh = _single()
    np.testing.assert_allclose(twod.element_mass_2d(mesh, p, p + 2)[0], _kron2(M1, M1), atol=1e-14)
    np.testing.assert_allclose(twod.element_stiffness_2d(mesh, p, p + 2)[0],
                               _kron2(K1, M1) + _kron2(M1, K1), atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_affine_element_stiffness_exact(p):
    """K = det A sum_ab (A^-1 A^-T)_ab S_ab with S_00 = K1 x M1, S_11 = M1 x K1,
    S_01 = C^T x C (exact 1D integrals)."""
    rng = np.random.default_rng(7 + p)
    A = np.eye(2) + 0.3 * rng.normal(size=(2, 2))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    M1, K1, C = _exact_1d(p)
    G = np.linalg.inv(A) @ np.linalg.inv(A).T
    S00, S11 = _kron2(K1, M1), _kron2(M1, K1)
    S01 = _kron2(C.T, C)      # int dphi_i/dx dphi_j/dy
    want = np.linalg.det(A) * (G[0, 0] * S00 + G[1, 1] * S11 + G[0, 1] * (S01 + S01.T))
    got = twod.element_stiffness_2d(_single(A), p, p + 2)[0]
    np.testing.assert_allclose(got, want, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("p", [1, 2, 3])
def test_constants_and_area(p):
    mesh = synth.quad_lattice(4, 0.15, seed=3, rotate_seed=4)
    S, K, M = _matrices(mesh, p, synth.lognormal_iid(16, p + 2, 1.0, seed=5, dim=2))
    one = np.ones(S.ndofs)
    assert np.abs(K @ one).max() < 1e-12 * abs(K).max()
    assert abs(one @ (M @ one) - 1.0) < 1e-13


@pytest.mark.parametrize("p", [1, 2])
def test_linear_patch(p):
    mesh = synth.quad_lattice(4, 0.2, seed=6, rotate_seed=7)
    S, K, _ = _matrices(mesh, p)
    X = S.dof_coordinates()
    u = 1.0 + 2.0 * X[:, 0] - 3.0 * X[:, 1]
    Kc, bc = oracle.constrain(K, np.zeros(S.ndofs), S.boundary, g=np.where(S.boundary, u, 0.0))
    x = spla.spsolve(Kc.tocsc(), bc)
    np.testing.assert_allclose(x, u, atol=1e-11)


def test_spd_after_elimination():
    mesh = synth.quad_lattice(3, 0.1, seed=8)
    S, K, _ = _matrices(mesh, 2)
    Kc, _ = oracle.constrain(K, np.zeros(S.ndofs), S.boundary)
    assert np.linalg.eigvalsh(Kc.toarray()).min() > 0
    assert (np.abs(np.linalg.eigvalsh(K.toarray())) < 1e-10).sum() == 1


@pytest.mark.parametrize("p", [1, 2])
def test_l2_convergence_rate(p):
    errs = []
    for n in (4, 8):
        mesh = synth.quad_lattice(n, 0.05, seed=9)
        S, K, _ = _matrices(mesh, p)
        b = oracle.forms.assemble_vector(S, twod.element_load_2d(mesh, p, p + 2, synth.sine_source))
        Kc, bc = oracle.constrain(K, b, S.boundary)
        u = spla.spsolve(Kc.tocsc(), bc)
        errs.append(twod.l2_error_2d(S, u, synth.sine_solution))
    rate = np.log2(errs[0] / errs[1])
    assert rate > p + 0.7, (errs, rate)


def test_rotated_vertex_lists_give_the_same_operator():
    a = synth.quad_lattice(3, 0.1, seed=10)
    b = synth.quad_lattice(3, 0.1, seed=10, rotate_seed=11)
    Sa, Ka, _ = _matrices(a, 3)
    Sb, Kb, _ = _matrices(b, 3)
    perm = match_by_coords(Sa.dof_coordinates(), Sb.dof_coordinates())
    Kb = Kb.toarray()[np.ix_(perm, perm)]
    assert np.abs(Ka.toarray() - Kb).max() < 1e-12 * np.abs(Kb).max()
    assert np.array_equal(Sa.boundary, Sb.boundary[perm])
