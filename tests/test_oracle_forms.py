"""Pins for the oracle's element matrices, assembly and boundary treatment (CPU only).

What fixes the expected values here is not the oracle's own code:
* exact 1D integrals of Lagrange polynomials built from a Vandermonde solve and
  integrated symbolically (numpy.polynomial), tensorised with Kronecker products;
* textbook 1D P1/P2 element matrices;
* the energy identity for linear functions, u^T K v = (c . d) * vol(E), which
  holds on any element whose map lies in the discrete space;
* the paper's 2D diffusion setup formula (adjugate form, "GPU Acceleration");
* volume = 1^T M 1 = 1 on the unit cube, K 1 = 0, the spectrum by brute force.
A few mutation tests show that plausible mistakes fail these pins.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import forms
from oracle.forms import assemble_vector
from oracle.quadrature import gauss_lobatto


def _lagrange_polys(nodes):
    """Lagrange polynomials via a Vandermonde solve (independent of the oracle)."""
    n = len(nodes)
    V = np.vander(nodes, n, increasing=True)
    C = np.linalg.solve(V, np.eye(n))
    return [np.polynomial.Polynomial(C[:, j]) for j in range(n)]


def _exact_1d(p):
    """Exact 1D matrices on [0,1]: mass, stiffness, and C[i,j] = int phi_i' phi_j."""
    L = _lagrange_polys(gauss_lobatto(p + 1))
    def integ(poly):
        P = poly.integ()
        return P(1.0) - P(0.0)
    M = np.array([[integ(a * b) for b in L] for a in L])
    K = np.array([[integ(a.deriv() * b.deriv()) for b in L] for a in L])
    C = np.array([[integ(a.deriv() * b) for b in L] for a in L])
    return M, K, C


def _kron3(t1, t2, t3):
    # lexicographic dof index i1 + D*(i2 + D*i3): the first axis varies fastest
    return np.kron(t3, np.kron(t2, t1))


def _single_element(A=None, c=None):
    verts = synth.HEX_CORNERS.astype(np.float64)
    if A is not None:
        verts = verts @ np.asarray(A).T + (0 if c is None else np.asarray(c))
    return {"vertices": verts, "hex": np.arange(8)[None, :], "geom_order": 1, "geom_nodes": None}


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_unit_cube_element_matrices_exact(p):
    M1, K1, _ = _exact_1d(p)
    mesh = _single_element()
    Me = forms.element_mass(mesh, p, p + 2)[0]
    Ke = forms.element_stiffness(mesh, p, p + 2)[0]
    np.testing.assert_allclose(Me, _kron3(M1, M1, M1), atol=1e-14)
    expected_K = _kron3(K1, M1, M1) + _kron3(M1, K1, M1) + _kron3(M1, M1, K1)
    np.testing.assert_allclose(Ke, expected_K, atol=1e-13)


def test_textbook_1d_matrices():
    M1, K1, _ = _exact_1d(1)
    np.testing.assert_allclose(M1, [[1 / 3, 1 / 6], [1 / 6, 1 / 3]], atol=1e-15)
    np.testing.assert_allclose(K1, [[1, -1], [-1, 1]], atol=1e-14)
    M2, K2, _ = _exact_1d(2)
    np.testing.assert_allclose(M2, np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30, atol=1e-14)
    np.testing.assert_allclose(K2, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_affine_element_stiffness_exact(p):
    """General affine map: K = det A * sum_ab (A^-1 A^-T)_ab S_ab, S from exact 1D integrals."""
    rng = np.random.default_rng(3 + p)
    A = np.eye(3) + 0.3 * rng.normal(size=(3, 3))
    assert np.linalg.det(A) > 0
    M1, K1, C1 = _exact_1d(p)
    Ainv = np.linalg.inv(A)
    G = Ainv @ Ainv.T
    Kexp = np.zeros(((p + 1) ** 3,) * 2)
    for a in range(3):
        for b in range(3):
            t = []
            for d in range(3):
                if d == a and d == b:
                    t.append(K1)
                elif d == a:
                    t.append(C1)
                elif d == b:
                    t.append(C1.T)
                else:
                    t.append(M1)
            Kexp += G[a, b] * _kron3(*t)
    Kexp *= np.linalg.det(A)
    Ke = forms.element_stiffness(_single_element(A, [0.2, -0.1, 0.4]), p, p + 2)[0]
    np.testing.assert_allclose(Ke, Kexp, atol=1e-12 * np.abs(Kexp).max())


def _linear_energy_check(mesh, p, q1d, coeff=None):
    s = oracle.H1Space(mesh, p)
    K = oracle.assemble(s, forms.element_stiffness(mesh, p, q1d, coeff))
    pts, w = forms.quadrature_points(q1d)
    _, J = oracle.map_points(mesh, pts)
    wdet = w[None, :] * np.linalg.det(J) * (1.0 if coeff is None else coeff)
    X = s.dof_coordinates()
    rng = np.random.default_rng(11)
    c, d = rng.normal(size=3), rng.normal(size=3)
    u, v = X @ c, X @ d
    return v @ (K @ u), np.dot(c, d) * wdet.sum()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_linear_energy_identity_jittered(p):
    mesh = synth.hex_lattice(3, 0.1, seed=2)
    got, want = _linear_energy_check(mesh, p, p + 2)
    assert abs(got - want) < 1e-12 * abs(want)


def test_linear_energy_identity_with_coefficient():
    mesh = synth.hex_lattice(2, 0.1, seed=4)
    kappa = synth.lognormal_iid(8, 5, 1.0, seed=3)
    got, want = _linear_energy_check(mesh, 3, 5, kappa)
    assert abs(got - want) < 1e-12 * abs(want)


@pytest.mark.parametrize("p", [2, 3])
def test_linear_energy_identity_q2_warped(p):
    mesh = synth.q2_warped_lattice(2, 0.05)
    got, want = _linear_energy_check(mesh, p, p + 2)
    assert abs(got - want) < 1e-12 * abs(want)


def test_paper_2d_setup_formula():
    """2D quadrature-point operator vs the adjugate form of the paper's listing."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        J = np.eye(2) + 0.4 * rng.normal(size=(2, 2))
        if np.linalg.det(J) <= 0:
            J[:, 0] *= -1
        W, alpha = rng.uniform(0.1, 1.0), rng.uniform(0.5, 2.0)
        J11, J21, J12, J22 = J[0, 0], J[1, 0], J[0, 1], J[1, 1]
        c = alpha * W / (J11 * J22 - J21 * J12)
        Y0 = c * (J12 * J12 + J22 * J22)
        Y1 = -c * (J12 * J11 + J22 * J21)
        Y2 = c * (J11 * J11 + J21 * J21)
        D = forms.qpoint_diffusion_operator(J, W, alpha)
        np.testing.assert_allclose([D[0, 0], D[0, 1], D[1, 0], D[1, 1]], [Y0, Y1, Y1, Y2], rtol=1e-13)


@pytest.mark.parametrize("mesh_kind", ["jitter", "q2"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_volume_and_constants(mesh_kind, p):
    mesh = synth.hex_lattice(3, 0.1, seed=1) if mesh_kind == "jitter" else synth.q2_warped_lattice(3)
    q1d = max(p + 2, 4)
    s = oracle.H1Space(mesh, p)
    M = oracle.assemble(s, forms.element_mass(mesh, p, q1d))
    K = oracle.assemble(s, forms.element_stiffness(mesh, p, q1d))
    one = np.ones(s.ndofs)
    assert abs(one @ (M @ one) - 1.0) < 1e-13
    assert np.abs(K @ one).max() < 1e-12
    # load of f = 1 integrates to the volume; of f = x to 1/2
    b1 = assemble_vector(s, forms.element_load(mesh, p, q1d, lambda x: np.ones(x.shape[:-1])))
    bx = assemble_vector(s, forms.element_load(mesh, p, q1d, lambda x: x[..., 0]))
    assert abs(b1.sum() - 1.0) < 1e-13
    assert abs(bx.sum() - 0.5) < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_spectrum_brute_force(p):
    mesh = synth.hex_lattice(2, 0.1, seed=9)
    s = oracle.H1Space(mesh, p)
    K = oracle.assemble(s, forms.element_stiffness(mesh, p, p + 2)).toarray()
    M = oracle.assemble(s, forms.element_mass(mesh, p, p + 2)).toarray()
    assert np.abs(K - K.T).max() < 1e-13
    ev = np.linalg.eigvalsh(K)
    assert abs(ev[0]) < 1e-12 * ev[-1] and ev[1] > 1e-6 * ev[-1]      # nullity exactly 1
    assert np.linalg.eigvalsh(M)[0] > 0
    Kc, _ = oracle.constrain(oracle.assemble(s, forms.element_stiffness(mesh, p, p + 2)),
                             np.zeros(s.ndofs), s.boundary)
    assert np.linalg.eigvalsh(Kc.toarray())[0] > 0


@pytest.mark.parametrize("case", [("jitter", 1), ("jitter", 2), ("q2", 2), ("q2", 3)])
def test_linear_patch(case):
    kind, p = case
    mesh = synth.hex_lattice(3, 0.1, seed=6) if kind == "jitter" else synth.q2_warped_lattice(2)
    s = oracle.H1Space(mesh, p)
    K = oracle.assemble(s, forms.element_stiffness(mesh, p, p + 2))
    X = s.dof_coordinates()
    g = synth.linear_patch(X)
    Kc, bc = oracle.constrain(K, np.zeros(s.ndofs), s.boundary, g)
    x = spla.spsolve(Kc.tocsc(), bc)
    assert np.abs(x - g).max() < 1e-11


@pytest.mark.parametrize("p,ns", [(1, (4, 8, 16)), (2, (2, 4, 8)), (3, (2, 4, 8))])
def test_l2_convergence_rate(p, ns):
    errs = []
    for n in ns:
        mesh = synth.hex_lattice(n, 0.1, seed=7)
        s = oracle.H1Space(mesh, p)
        K = oracle.assemble(s, forms.element_stiffness(mesh, p, p + 2))
        b = assemble_vector(s, forms.element_load(mesh, p, p + 2, synth.sine_source))
        Kc, bc = oracle.constrain(K, b, s.boundary)
        x = spla.spsolve(Kc.tocsc(), bc)
        errs.append(oracle.l2_error(s, x, synth.sine_solution))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert abs(rates[-1] - (p + 1)) < 0.3, rates


# ---- mutation tests: plausible mistakes must fail the pins above ----------------

def test_mutant_transposed_metric_fails(monkeypatch):
    orig = forms.qpoint_diffusion_operator

    def transposed(J, weight, coeff=1.0):
        return orig(np.swapaxes(J, -1, -2), weight, coeff)
    monkeypatch.setattr(forms, "qpoint_diffusion_operator", transposed)
    mesh = synth.hex_lattice(2, 0.1, seed=2)
    got, want = _linear_energy_check(mesh, 2, 4)
    assert abs(got - want) > 1e-6 * abs(want)


def test_mutant_short_quadrature_fails():
    # integrating the unit-cube stiffness with too few points breaks the exact pin
    M1, K1, _ = _exact_1d(3)
    Ke = forms.element_stiffness(_single_element(), 3, 2)[0]
    expected_K = _kron3(K1, M1, M1) + _kron3(M1, K1, M1) + _kron3(M1, M1, K1)
    assert np.abs(Ke - expected_K).max() > 1e-6


def test_patch_rows_equal_whole_mesh_rows():
    """The sampled-row oracle of the full-size parity tests: rows of the constrained
    operator from a 3x3x3 element block equal the rows of the whole-mesh matrix
    (interior, face, edge and corner elements; diffusion and mass)."""
    from tests._common import OracleProblem, patch_rows
    n, p = 5, 2
    mesh = synth.hex_lattice(n, 0.08, seed=7)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=8)
    ref = OracleProblem(mesh, p, coeff=kappa, rho=kappa)
    x = synth.hash_normal(ref.coords, seed=9)
    for kind, A in (("diffusion", ref.Kc), ("mass", ref.Mc)):
        y = A @ x
        for c in (0, E - 1, 12, 62, 2 + n * (2 + n * 2)):
            yo, Xo = patch_rows(mesh, kappa, p, c, kind, seed=9)
            idx = [int(np.argmin(np.abs(ref.coords - xo).sum(axis=1))) for xo in Xo]
            assert np.abs(ref.coords[idx] - Xo).max() < 1e-12
            np.testing.assert_allclose(yo, y[idx], rtol=1e-12, atol=1e-12 * np.abs(y).max())


@pytest.mark.parametrize("p", [1, 2, 3])
def test_convection_affine_element_exact(p):
    """Affine map x = A xhat, constant beta: C_E = det A sum_b (A^-1 beta)_b S_b with
    S_b the tensor product of exact 1D integrals (C^T along axis b, M elsewhere)."""
    rng = np.random.default_rng(11 + p)
    A = np.eye(3) + 0.3 * rng.normal(size=(3, 3))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    beta = np.array([0.7, -1.3, 0.4])
    M1, _, C1 = _exact_1d(p)
    g = np.linalg.solve(A, beta)
    # C1[i, j] = int phi_i' phi_j, so int phi_i phi_j' = C1[j, i]
    S = [_kron3(C1.T, M1, M1), _kron3(M1, C1.T, M1), _kron3(M1, M1, C1.T)]
    want = np.linalg.det(A) * sum(g[b] * S[b] for b in range(3))
    got = forms.element_convection(_single_element(A), p, p + 2, beta)[0]
    np.testing.assert_allclose(got, want, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("p", [1, 2, 3])
def test_convection_constants_and_skew_symmetry(p):
    """C 1 = 0; for a divergence-free velocity C + C^T vanishes on functions that are
    zero on the boundary (integration by parts), on jittered, rotated meshes."""
    mesh = synth.hex_lattice(3, 0.1, seed=4, rotate_seed=5)
    S = oracle.H1Space(mesh, p)
    vel = lambda x: np.stack([x[..., 1] - 0.5, 0.5 - x[..., 0], 0.3 + 0.0 * x[..., 2]], axis=-1)
    C = oracle.assemble(S, forms.element_convection(mesh, p, p + 2, vel)).toarray()
    assert np.abs(C @ np.ones(S.ndofs)).max() < 1e-12 * np.abs(C).max()
    free = ~S.boundary
    Cf = C[np.ix_(free, free)]
    # the velocity is linear, so every rule of q1d = p + 2 integrates it exactly on
    # affine maps only; jittered trilinear maps leave a quadrature error
    assert np.abs(Cf + Cf.T).max() < 5e-3 * np.abs(Cf).max()
    flat = synth.hex_lattice(3, 0.0, rotate_seed=5)
    S0 = oracle.H1Space(flat, p)
    C0 = oracle.assemble(S0, forms.element_convection(flat, p, p + 2, vel)).toarray()
    f0 = ~S0.boundary
    C0f = C0[np.ix_(f0, f0)]
    assert np.abs(C0f + C0f.T).max() < 1e-12 * np.abs(C0f).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_gradient_of_linear_functions_and_convection(p):
    """grad of a + b.x is b everywhere: G_c u = b_c M 1 exactly (the same rule as the
    mass matrix); sum_c beta_c G_c is the convection matrix of a constant beta."""
    mesh = synth.hex_lattice(3, 0.15, seed=6, rotate_seed=7)
    S = oracle.H1Space(mesh, p)
    kappa = synth.lognormal_iid(mesh["hex"].shape[0], p + 2, 1.0, seed=8)
    Ge = forms.element_gradient(mesh, p, p + 2, kappa)
    G = [oracle.assemble(S, Ge[:, c]) for c in range(3)]
    M = oracle.assemble(S, forms.element_mass(mesh, p, p + 2, kappa))
    X = S.dof_coordinates()
    bvec = np.array([0.7, -1.2, 2.0])
    u = 0.3 + X @ bvec
    m1 = M @ np.ones(S.ndofs)
    for c in range(3):
        np.testing.assert_allclose(G[c] @ u, bvec[c] * m1, atol=1e-12 * np.abs(m1).max())
    beta = np.array([0.4, 1.1, -0.6])
    Gu = forms.element_gradient(mesh, p, p + 2)
    C = oracle.assemble(S, forms.element_convection(mesh, p, p + 2, beta)).toarray()
    Gb = sum(beta[c] * oracle.assemble(S, Gu[:, c]).toarray() for c in range(3))
    assert np.abs(Gb - C).max() <= 1e-12 * np.abs(C).max()


@pytest.mark.parametrize("p", [1, 2])
def test_gradient_affine_element_exact(p):
    """Affine map, constant coefficient: G_c = det A sum_b (A^-1)_bc S_b (exact 1D integrals)."""
    rng = np.random.default_rng(21 + p)
    A = np.eye(3) + 0.3 * rng.normal(size=(3, 3))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    M1, _, C1 = _exact_1d(p)
    S = [_kron3(C1.T, M1, M1), _kron3(M1, C1.T, M1), _kron3(M1, M1, C1.T)]
    Ainv = np.linalg.inv(A)
    got = forms.element_gradient(_single_element(A), p, p + 2)[0]
    for c in range(3):
        want = np.linalg.det(A) * sum(Ainv[b, c] * S[b] for b in range(3))
        np.testing.assert_allclose(got[c], want, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("p", [1, 2, 3])
def test_divergence_of_linear_vector_fields(p):
    """u = A x + b lies in the space and div u = tr A, so sum_c V_c u_c = tr(A) M 1
    exactly (M the kappa-weighted mass matrix, the same rule)."""
    mesh = synth.hex_lattice(3, 0.15, seed=16, rotate_seed=17)
    S = oracle.H1Space(mesh, p)
    kappa = synth.lognormal_iid(mesh["hex"].shape[0], p + 2, 1.0, seed=18)
    Ve = forms.element_divergence(mesh, p, p + 2, kappa)
    V = [oracle.assemble(S, Ve[:, c]) for c in range(3)]
    M = oracle.assemble(S, forms.element_mass(mesh, p, p + 2, kappa))
    X = S.dof_coordinates()
    A = np.array([[0.3, -1.1, 0.4], [0.9, 1.7, -0.2], [0.5, 0.8, -2.3]])
    u = X @ A.T + np.array([0.2, -0.7, 1.3])
    m1 = M @ np.ones(S.ndofs)
    got = sum(V[c] @ u[:, c] for c in range(3))
    np.testing.assert_allclose(got, np.trace(A) * m1, atol=1e-12 * np.abs(m1).max())
    # a field with zero divergence, u = (y, -x, 0) (rotation), gives zero
    rot = np.stack([X[:, 1], -X[:, 0], np.zeros(S.ndofs)], axis=1)
    assert np.abs(sum(V[c] @ rot[:, c] for c in range(3))).max() < 1e-12 * np.abs(m1).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_divergence_integration_by_parts(p):
    """For u vanishing on the boundary, (div u, q) = -(u, grad q).  On trilinear
    elements the integrand of int d(u_c q)/dx_c is a polynomial of degree <= 2p + 2
    per reference direction, which the (p + 2)-point rule integrates exactly: the
    divergence matrices equal minus the transposed gradient matrices on columns of
    interior dofs, on jittered meshes too."""
    mesh = synth.hex_lattice(3, 0.15, seed=26, rotate_seed=27)
    S = oracle.H1Space(mesh, p)
    Ve = forms.element_divergence(mesh, p, p + 2)
    Ge = forms.element_gradient(mesh, p, p + 2)
    free = ~S.boundary
    for c in range(3):
        V = oracle.assemble(S, Ve[:, c]).toarray()
        G = oracle.assemble(S, Ge[:, c]).toarray()
        lhs = V[:, free]
        rhs = -G.T[:, free]
        assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(lhs).max()


@pytest.mark.parametrize("p", [1, 2])
def test_divergence_affine_element_exact(p):
    """Affine map, constant coefficient: V_c = det A sum_b (A^-1)_bc S_b (exact 1D integrals)."""
    rng = np.random.default_rng(41 + p)
    A = np.eye(3) + 0.3 * rng.normal(size=(3, 3))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    M1, _, C1 = _exact_1d(p)
    S = [_kron3(C1.T, M1, M1), _kron3(M1, C1.T, M1), _kron3(M1, M1, C1.T)]
    Ainv = np.linalg.inv(A)
    got = forms.element_divergence(_single_element(A), p, p + 2)[0]
    for c in range(3):
        want = np.linalg.det(A) * sum(Ainv[b, c] * S[b] for b in range(3))
        np.testing.assert_allclose(got[c], want, atol=1e-12 * np.abs(want).max())


def _elasticity_global(mesh, p, lam, mu):
    S = oracle.H1Space(mesh, p)
    Ke = forms.element_elasticity(mesh, p, p + 2, lam, mu)
    E, nd = Ke.shape[0], Ke.shape[2]
    V = forms.vector_space(S)
    return S, V, oracle.assemble(V, Ke.reshape(E, 3 * nd, 3 * nd))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_elasticity_rigid_modes_and_patch(p):
    """The six rigid-body fields (translations, infinitesimal rotations w x X) have zero
    strain and lie in the space: K u = 0 exactly for point-varying lambda, mu.  For a
    linear field and constant lambda, mu the stress is constant and K u vanishes on
    interior rows (the integrand of int sigma : grad v has degree <= p + 2 per reference
    direction on trilinear elements)."""
    mesh = synth.hex_lattice(3, 0.15, seed=31, rotate_seed=32)
    E = mesh["hex"].shape[0]
    lam = synth.lognormal_iid(E, p + 2, 0.5, seed=33)
    mu = synth.lognormal_iid(E, p + 2, 0.5, seed=34)
    S, V, K = _elasticity_global(mesh, p, lam, mu)
    X = S.dof_coordinates()
    scale = np.abs(K).max()
    modes = [np.tile(e, (S.ndofs, 1)) for e in np.eye(3)]
    for w in np.eye(3):
        modes.append(np.cross(w, X))
    for u in modes:
        assert np.abs(K @ u.T.ravel()).max() <= 1e-11 * scale
    S1, V1, K1 = _elasticity_global(mesh, p, 1.7, 0.6)
    A = np.array([[0.3, -1.1, 0.4], [0.9, 1.7, -0.2], [0.5, 0.8, -2.3]])
    u = (X @ A.T + 0.3).T.ravel()
    r = K1 @ u
    assert np.abs(r[~V1.boundary]).max() <= 1e-11 * np.abs(K1).max()
    assert np.abs(r[V1.boundary]).max() > 1e-3 * np.abs(K1).max()


@pytest.mark.parametrize("p", [1, 2])
def test_elasticity_parts_against_gradient_and_diffusion(p):
    """lambda part (mu = 0): for u = A x + b the load is tr(A) int d_c phi_i = tr(A)
    (G_c^T 1)_i with the gradient matrices.  mu part (lambda = 0): the diagonal blocks
    sum to 4 times the diffusion stiffness (sum_c (delta_cc grad.grad + d_c d_c) = 3 L + L)."""
    mesh = synth.hex_lattice(2, 0.15, seed=36, rotate_seed=37)
    E = mesh["hex"].shape[0]
    kap = synth.lognormal_iid(E, p + 2, 0.5, seed=38)
    S = oracle.H1Space(mesh, p)
    X = S.dof_coordinates()
    A = np.array([[0.3, -1.1, 0.4], [0.9, 1.7, -0.2], [0.5, 0.8, -2.3]])
    u = (X @ A.T + np.array([0.1, 0.2, -0.3])).T.ravel()
    _, _, Kl = _elasticity_global(mesh, p, kap, 0.0)
    Ge = forms.element_gradient(mesh, p, p + 2, kap)
    ones = np.ones(S.ndofs)
    want = np.concatenate([np.trace(A) * (oracle.assemble(S, Ge[:, c]).T @ ones) for c in range(3)])
    np.testing.assert_allclose(Kl @ u, want, atol=1e-12 * np.abs(want).max())
    Km = forms.element_elasticity(mesh, p, p + 2, 0.0, kap)
    L = forms.element_stiffness(mesh, p, p + 2, kap)
    np.testing.assert_allclose(sum(Km[:, c, :, c, :] for c in range(3)), 4.0 * L,
                               atol=1e-12 * np.abs(L).max())


@pytest.mark.parametrize("p", [1, 2])
def test_elasticity_affine_element_exact(p):
    """Affine map x = A xhat, constant lambda, mu: with S_ab[i, j] = int dhat_a phi_i dhat_b phi_j
    (Kronecker products of exact 1D integrals) and Ai = A^-1,
    K[c,i,d,j] = det A sum_ab S_ab [lambda Ai_ac Ai_bd + mu (delta_cd (Ai Ai^T)_ab + Ai_ad Ai_bc)]."""
    rng = np.random.default_rng(51 + p)
    A = np.eye(3) + 0.3 * rng.normal(size=(3, 3))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    lam, mu = 1.3, 0.7
    M1, K1, C1 = _exact_1d(p)
    Sab = {}
    for a in range(3):
        for b in range(3):
            t = []
            for d in range(3):
                if d == a and d == b:
                    t.append(K1)
                elif d == a:
                    t.append(C1)
                elif d == b:
                    t.append(C1.T)
                else:
                    t.append(M1)
            Sab[a, b] = _kron3(*t)
    Ai = np.linalg.inv(A)
    G = Ai @ Ai.T
    got = forms.element_elasticity(_single_element(A, [0.1, 0.0, -0.2]), p, p + 2, lam, mu)[0]
    for c in range(3):
        for d in range(3):
            want = np.linalg.det(A) * sum(
                Sab[a, b] * (lam * Ai[a, c] * Ai[b, d]
                             + mu * ((c == d) * G[a, b] + Ai[a, d] * Ai[b, c]))
                for a in range(3) for b in range(3))
            np.testing.assert_allclose(got[c, :, d, :], want, atol=1e-12 * np.abs(want).max())


def test_elasticity_null_space_dimension():
    """Symmetric positive semidefinite with exactly the six rigid-body modes as kernel."""
    mesh = synth.hex_lattice(2, 0.15, seed=41, rotate_seed=42)
    E = mesh["hex"].shape[0]
    _, _, K = _elasticity_global(mesh, 1, synth.lognormal_iid(E, 3, 0.5, seed=43),
                                 synth.lognormal_iid(E, 3, 0.5, seed=44))
    K = K.toarray()
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    tol = 1e-10 * ev[-1]
    assert ev[0] > -tol and int((np.abs(ev) <= tol).sum()) == 6
