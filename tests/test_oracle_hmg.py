"""Pins for the mesh-size (h-) multigrid part of the multigrid oracle (CPU only):
uniform refinement and the interpolation from a coarse mesh to its refinement."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import forms, mlp, pmg
from oracle.basis import tensor_points, tensor_weights
from oracle.quadrature import gauss_legendre


def _lin(X):
    return 1.0 + 2.0 * X[:, 0] - X[:, 1] + 3.0 * X[:, 2]


def _quad(X):
    return X[:, 0] * X[:, 1] + X[:, 2] ** 2 - 0.5 * X[:, 1] * X[:, 2]


def _volumes(mesh, q=4):
    x, w = gauss_legendre(q)
    _, J = oracle.map_points(mesh, tensor_points(x))
    return np.linalg.det(J) @ tensor_weights(w)


MESHES = {
    "jittered": lambda: synth.hex_lattice((2, 3, 2), 0.2, seed=3),
    "rotated": lambda: synth.hex_lattice(2, 0.15, seed=4, rotate_seed=5),
    "quadratic": lambda: synth.q2_warped_lattice(2, 0.05),
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_children_carry_the_parent_map(name):
    """Each child's own geometry (its vertices, or its 27 nodes) maps its reference
    points where the parent's map sends the octant's points, so the children tile the
    parent: their volumes add up to the parent's, and no child is inverted."""
    mesh = MESHES[name]()
    fine = pmg.refine(mesh)
    E = mesh["hex"].shape[0]
    assert fine["hex"].shape == (8 * E, 8)
    x, _ = gauss_legendre(3)
    ref = tensor_points(x)
    xf, Jf = oracle.map_points(fine, ref)
    for o in range(8):
        off = np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1], dtype=float)
        xp, _ = oracle.map_points(mesh, (off + ref) / 2.0)
        np.testing.assert_allclose(xf[o::8], xp, rtol=0, atol=1e-13)
    assert np.linalg.det(Jf).min() > 0
    np.testing.assert_allclose(_volumes(fine).reshape(E, 8).sum(axis=1), _volumes(mesh),
                               rtol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_refined_lattice_is_the_lattice_twice_as_fine(p):
    """Refining the n^3 lattice gives the (2n)^3 lattice: the same vertex set, a
    conforming mesh (H1 dof and boundary counts of the finer lattice), also when the
    coarse elements' vertex lists are rotated."""
    for rot in (None, 9):
        coarse = synth.hex_lattice(2, 0.0, rotate_seed=rot)
        fine = pmg.refine(coarse)
        flat = synth.hex_lattice(4, 0.0)
        a = np.round(fine["vertices"], 12)
        b = np.round(flat["vertices"], 12)
        assert a.shape == b.shape
        assert np.array_equal(a[np.lexsort(a.T)], b[np.lexsort(b.T)])
        S = oracle.H1Space(fine, p)
        m = 4 * p + 1
        assert S.ndofs == m ** 3
        assert int(S.boundary.sum()) == m ** 3 - (m - 2) ** 3


@pytest.mark.parametrize("pc,pf", [(1, 1), (1, 2), (2, 2), (2, 3), (3, 3)])
def test_h_interpolation_reproduces_coarse_functions(pc, pf):
    """Physical linear functions are in every order's space on trilinear meshes; the
    children's maps are the parent's, so their coarse nodal values must prolongate to
    their fine nodal values; on affine meshes also quadratics for pc >= 2."""
    mesh = synth.hex_lattice((2, 2, 1), 0.15, seed=3, rotate_seed=4)
    fine = pmg.refine(mesh)
    P = pmg.h_interpolation(mesh, fine, pc, pf, free_only=False)
    Xc = oracle.H1Space(mesh, pc).dof_coordinates()
    Xf = oracle.H1Space(fine, pf).dof_coordinates()
    np.testing.assert_allclose(P @ _lin(Xc), _lin(Xf), rtol=0, atol=1e-13)
    np.testing.assert_allclose(P @ np.ones(Xc.shape[0]), 1.0, rtol=0, atol=1e-14)
    if pc >= 2:
        flat = synth.hex_lattice((2, 1, 2), 0.0, rotate_seed=5)
        ff = pmg.refine(flat)
        P = pmg.h_interpolation(flat, ff, pc, pf, free_only=False)
        Xc = oracle.H1Space(flat, pc).dof_coordinates()
        Xf = oracle.H1Space(ff, pf).dof_coordinates()
        np.testing.assert_allclose(P @ _quad(Xc), _quad(Xf), rtol=0, atol=1e-13)


@pytest.mark.parametrize("pc,pf", [(1, 1), (1, 2), (2, 2), (2, 3), (3, 3)])
def test_h_galerkin_identity_on_affine_meshes(pc, pf):
    """The refined space contains the coarse one, and with affine elements and a
    constant coefficient both rules integrate exactly, so P^T A_f P is the coarse
    matrix.  A wrong octant, a transposed table or a misplaced child breaks this."""
    mesh = synth.hex_lattice((2, 2, 1), 0.0, rotate_seed=7)
    fine = pmg.refine(mesh)
    P = pmg.h_interpolation(mesh, fine, pc, pf, free_only=False)
    Sc, Sf = oracle.H1Space(mesh, pc), oracle.H1Space(fine, pf)
    for make in (forms.element_stiffness, forms.element_mass):
        Af = oracle.assemble(Sf, make(fine, pf, pf + 2, 2.5))
        Ac = oracle.assemble(Sc, make(mesh, pc, pc + 2, 2.5)).toarray()
        G = (P.T @ Af @ P).toarray()
        assert np.abs(G - Ac).max() <= 1e-12 * np.abs(Ac).max()


def test_level_coefficient_is_the_mean_over_descendants():
    c = np.arange(1.0, 1.0 + 16 * 8).reshape(16, 8)   # 16 finest elements, 2^3 points
    out = pmg.level_coefficient(c, 2, 3)              # two coarse elements, 3^3 points
    assert out.shape == (2, 27)
    np.testing.assert_allclose(out[:, 0], [c[:8].mean(), c[8:].mean()])
    np.testing.assert_allclose(out, out[:, :1].repeat(27, axis=1))
    g = pmg.level_coefficient(np.exp(c / 50.0), 2, 1, "geometric")
    np.testing.assert_allclose(np.log(g[:, 0]), [c[:8].mean() / 50.0, c[8:].mean() / 50.0])


def _hp(meshes, plan, coeff=None):
    starts = [synth.hash_normal(oracle.H1Space(meshes[m], p).dof_coordinates(), seed=40 + l)
              for l, (m, p) in enumerate(plan)]
    return pmg.build_hp_levels(meshes, plan, coeff, "arithmetic", starts)


def test_hp_two_level_cycle_is_symmetric_positive_definite():
    """Brute force: the matrix of b -> V(b) over an h-step with an exact coarse solve
    is SPD, and the two-grid error propagation contracts in the A-norm."""
    coarse = synth.hex_lattice(2, 0.1, seed=8)
    fine = pmg.refine(coarse)
    levels, _ = _hp([fine, coarse], [(0, 1), (1, 1)])
    n = levels[0]["A"].shape[0]
    V = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        V[:, j] = pmg.vcycle(levels, e, coarse_iters=None)
    assert np.abs(V - V.T).max() <= 1e-10 * np.abs(V).max()
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0
    A = levels[0]["A"].toarray()
    Ah = sla.sqrtm(A).real
    assert np.linalg.norm(Ah @ (np.eye(n) - V @ A) @ np.linalg.inv(Ah), 2) < 0.9


def test_hp_fcg_solves_and_beats_jacobi():
    """Orders then mesh sizes: p = 2 -> 1 on the fine mesh, then two h-steps."""
    m2 = synth.hex_lattice(2, 0.1, seed=6)
    m1 = pmg.refine(m2)
    m0 = pmg.refine(m1)
    E = m0["hex"].shape[0]
    kappa = synth.lognormal_iid(E, 4, 1.0, seed=5)
    levels, spaces = _hp([m0, m1, m2], [(0, 2), (0, 1), (1, 1), (2, 1)], kappa)
    A = levels[0]["A"]
    S = spaces[0]
    b = forms.assemble_vector(S, forms.element_load(m0, 2, 4, synth.sine_source))
    b[S.boundary] = 0.0
    x, k, _ = mlp.fcg(A, b, lambda r: pmg.vcycle(levels, r, coarse_iters=10), tol=1e-8)
    jac = oracle.pcg(A, b, A.diagonal(), tol=1e-8)
    xd = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
    assert 2 * k < jac["iters"], (k, jac["iters"])


def _two_grid_contraction(nc):
    coarse = synth.hex_lattice(nc, 0.1, seed=8)
    fine = pmg.refine(coarse)
    levels, spaces = _hp([fine, coarse], [(0, 1), (1, 1)])
    A = levels[0]["A"].toarray()
    free = ~spaces[0].boundary
    n = A.shape[0]
    V = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        V[:, j] = pmg.vcycle(levels, e, coarse_iters=None)
    Af, Vf = A[np.ix_(free, free)], V[np.ix_(free, free)]
    Ah = sla.sqrtm(Af).real
    return np.linalg.norm(Ah @ (np.eye(Af.shape[0]) - Vf @ Af) @ np.linalg.inv(Ah), 2)


def test_two_grid_contraction_does_not_grow_under_refinement():
    """The property that makes multigrid worth its levels: the A-norm contraction of the
    two-grid cycle (degree-2 Chebyshev smoothing, exact coarse solve) stays small and
    does not grow as the mesh is refined (coarse 2^3, 3^3, 4^3 elements at p = 1; about
    0.038 at each size)."""
    r = [_two_grid_contraction(nc) for nc in (2, 3, 4)]
    print("two-grid contraction", r)
    assert max(r) < 0.1
    assert max(r) < 1.2 * min(r)
