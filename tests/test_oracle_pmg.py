"""Pins for the order-multigrid oracle (CPU only)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla
from numpy.polynomial import chebyshev as npcheb

import oracle
import synth
from oracle import forms, mlp, pmg


def _lin(X):
    return 1.0 + 2.0 * X[:, 0] - X[:, 1] + 3.0 * X[:, 2]


def _quad(X):
    return X[:, 0] * X[:, 1] + X[:, 2] ** 2 - 0.5 * X[:, 1] * X[:, 2]


@pytest.mark.parametrize("pc,pf", [(1, 1), (1, 2), (1, 3), (2, 3), (2, 4), (3, 5)])
def test_interpolation_reproduces_coarse_functions(pc, pf):
    """Physical-space linear functions lie in every order's space on trilinear meshes,
    so interpolating their coarse nodal values must give their fine nodal values."""
    mesh = synth.hex_lattice((2, 2, 1), 0.15, seed=3, rotate_seed=4)
    P = pmg.interpolation(mesh, pc, pf, free_only=False)
    Xc = oracle.H1Space(mesh, pc).dof_coordinates()
    Xf = oracle.H1Space(mesh, pf).dof_coordinates()
    np.testing.assert_allclose(P @ _lin(Xc), _lin(Xf), rtol=0, atol=1e-13)
    np.testing.assert_allclose(P @ np.ones(Xc.shape[0]), 1.0, rtol=0, atol=1e-14)
    if pc >= 2:
        # on an affine mesh, functions of degree <= 2 per coordinate are in Q_pc
        flat = synth.hex_lattice((2, 1, 2), 0.0, rotate_seed=5)
        P = pmg.interpolation(flat, pc, pf, free_only=False)
        Xc = oracle.H1Space(flat, pc).dof_coordinates()
        Xf = oracle.H1Space(flat, pf).dof_coordinates()
        np.testing.assert_allclose(P @ _quad(Xc), _quad(Xf), rtol=0, atol=1e-13)


def test_interpolation_between_equal_orders_is_identity():
    mesh = synth.hex_lattice(2, 0.1, seed=1, rotate_seed=2)
    P = pmg.interpolation(mesh, 3, 3, free_only=False).toarray()
    np.testing.assert_allclose(P, np.eye(P.shape[0]), atol=1e-14)
    S = oracle.H1Space(mesh, 3)
    P0 = pmg.interpolation(mesh, 3, 3).toarray()
    np.testing.assert_allclose(P0, np.diag((~S.boundary).astype(float)), atol=1e-14)


@pytest.mark.parametrize("pc,pf", [(1, 2), (1, 3), (2, 3), (2, 4), (3, 3)])
def test_galerkin_identity_on_affine_meshes(pc, pf):
    """With affine elements and a constant coefficient both rules integrate exactly,
    so P^T A_f P is the coarse matrix itself.  A transposed or misplaced entry of P
    breaks this."""
    mesh = synth.hex_lattice((2, 2, 1), 0.0, rotate_seed=7)
    P = pmg.interpolation(mesh, pc, pf, free_only=False)
    Sc, Sf = oracle.H1Space(mesh, pc), oracle.H1Space(mesh, pf)
    for make in (forms.element_stiffness, forms.element_mass):
        Af = oracle.assemble(Sf, make(mesh, pf, pf + 2, 2.5))
        Ac = oracle.assemble(Sc, make(mesh, pc, pc + 2, 2.5)).toarray()
        G = (P.T @ Af @ P).toarray()
        assert np.abs(G - Ac).max() <= 1e-12 * np.abs(Ac).max()


def test_chebyshev_error_is_the_scaled_polynomial():
    """On A = diag(lambda) with D = I the error after m steps from x = 0 is
    T_m((theta - lambda)/delta) / T_m(theta/delta) times the initial error."""
    lam = np.linspace(0.05, 2.2, 40)
    A = np.diag(lam)
    rng = np.random.default_rng(3)
    e0 = rng.normal(size=lam.size)
    b = A @ e0
    lmax, lo, hi = 2.0, 0.3, 1.1
    theta, delta = 0.5 * (hi + lo) * lmax, 0.5 * (hi - lo) * lmax
    for m in (1, 2, 3, 5, 8):
        x = pmg.chebyshev(A, np.ones(lam.size), b, None, lmax, m, lo, hi)
        Tm = np.zeros(m + 1)
        Tm[m] = 1.0
        want = npcheb.chebval((theta - lam) / delta, Tm) / npcheb.chebval(theta / delta, Tm) * e0
        np.testing.assert_allclose(e0 - x, want, rtol=1e-10, atol=1e-12)


def test_chebyshev_from_a_guess_is_affine_in_the_guess():
    """x_m(x0) = x0 + S(b - A x0) with the same polynomial S as from zero."""
    mesh = synth.hex_lattice(2, 0.1, seed=2)
    levels, _ = pmg.build_levels(mesh, [2])
    A, d = levels[0]["A"], levels[0]["diag"]
    rng = np.random.default_rng(5)
    b, x0 = rng.normal(size=A.shape[0]), rng.normal(size=A.shape[0])
    x = pmg.chebyshev(A, d, b, x0, 2.0, 3)
    np.testing.assert_allclose(x, x0 + pmg.chebyshev(A, d, b - A @ x0, None, 2.0, 3), atol=1e-12)


def test_power_iteration_approaches_lambda_max_from_below():
    mesh = synth.hex_lattice(2, 0.1, seed=4)
    ref = oracle.H1Space(mesh, 2)
    A = oracle.constrain(oracle.assemble(ref, forms.element_stiffness(mesh, 2, 4)),
                         np.zeros(ref.ndofs), ref.boundary)[0]
    d = A.diagonal()
    lam_true = sla.eigh(A.toarray(), np.diag(d), eigvals_only=True).max()
    v0 = synth.hash_normal(ref.dof_coordinates(), seed=9)
    prev = 0.0
    for k in (1, 2, 5, 10, 40):
        lam = pmg.power_lmax(A, d, v0, k)
        assert lam <= lam_true * (1 + 1e-12)
        assert lam >= prev - 1e-13
        prev = lam
    assert abs(pmg.power_lmax(A, d, v0, 600) - lam_true) <= 1e-6 * lam_true


def test_element_mean_closed_forms():
    c = np.array([[1.0, 2.0, 4.0], [3.0, 3.0, 3.0]])
    np.testing.assert_allclose(pmg.element_mean(c, "arithmetic"), [7.0 / 3.0, 3.0])
    np.testing.assert_allclose(pmg.element_mean(c, "geometric"), [2.0, 3.0])
    np.testing.assert_allclose(pmg.element_mean(c, "harmonic"), [12.0 / 7.0, 3.0])


def _levels(mesh, orders, coeff=None, mean="arithmetic"):
    starts = [synth.hash_normal(oracle.H1Space(mesh, p).dof_coordinates(), seed=20 + p)
              for p in orders]
    return pmg.build_levels(mesh, orders, coeff, mean, starts)


def test_vcycle_with_the_fine_space_as_exact_coarse_level_is_the_inverse():
    mesh = synth.hex_lattice(2, 0.1, seed=6, rotate_seed=1)
    levels, spaces = _levels(mesh, [2, 2])
    A = levels[0]["A"]
    b = synth.hash_normal(spaces[0].dof_coordinates(), seed=3)
    b[spaces[0].boundary] = 0.0
    x = pmg.vcycle(levels, b, coarse_iters=None)
    xd = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


def test_two_level_cycle_is_symmetric_positive_definite():
    """Brute force: the matrix of b -> V(b) with an exact coarse solve."""
    mesh = synth.hex_lattice(2, 0.1, seed=8)
    levels, spaces = _levels(mesh, [3, 1])
    n = levels[0]["A"].shape[0]
    V = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        V[:, j] = pmg.vcycle(levels, e, coarse_iters=None)
    assert np.abs(V - V.T).max() <= 1e-10 * np.abs(V).max()
    ev = np.linalg.eigvalsh(0.5 * (V + V.T))
    assert ev.min() > 0
    # two-grid error propagation I - V A contracts in the A-norm
    A = levels[0]["A"].toarray()
    Ah = sla.sqrtm(A).real
    Einv = np.linalg.inv(Ah)
    assert np.linalg.norm(Ah @ (np.eye(n) - V @ A) @ Einv, 2) < 0.9


def test_pmg_fcg_beats_jacobi_pcg_and_solves():
    mesh = synth.hex_lattice(4, 0.1, seed=2)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, 6, 1.0, seed=5)
    levels, spaces = _levels(mesh, [4, 2, 1], kappa)
    A = levels[0]["A"]
    S = spaces[0]
    b = forms.assemble_vector(S, forms.element_load(mesh, 4, 6, synth.sine_source))
    b[S.boundary] = 0.0
    x, k, _ = mlp.fcg(A, b, lambda r: pmg.vcycle(levels, r, coarse_iters=10), tol=1e-8)
    jac = oracle.pcg(A, b, A.diagonal(), tol=1e-8)
    xd = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
    assert 3 * k < jac["iters"], (k, jac["iters"])
