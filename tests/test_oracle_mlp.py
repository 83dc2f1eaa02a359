"""Pins for the learned-preconditioner oracle (CPU only)."""
import numpy as np
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import forms, mlp
from tests._common import OracleProblem


def _params(seed=0, zero_last=False, i=10, h=12, o=6):
    return synth.mlp_init(i, h, o, seed=seed, zero_last=zero_last)


def test_backward_matches_finite_differences():
    P = _params(1)
    rng = np.random.default_rng(2)
    for k in P:
        P[k] = P[k] + 0.1 * rng.normal(size=P[k].shape)   # no dead units at zero bias
    X = rng.normal(size=(7, 10))
    W = rng.normal(size=(7, 6))
    out, cache = mlp.forward(P, X)
    G = mlp.backward(P, cache, W)          # gradient of sum(W * out)
    h = 1e-6
    for k in P:
        flat = P[k].ravel()
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            fp = np.sum(W * mlp.forward(P, X)[0])
            flat[idx] = old - h
            fm = np.sum(W * mlp.forward(P, X)[0])
            flat[idx] = old
            fd = (fp - fm) / (2 * h)
            assert abs(fd - G[k].ravel()[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_adam_closed_form_first_steps():
    # with constant gradient g, m_hat = g and v_hat = g^2: each step moves lr*g/(|g|+eps)
    P = {"w": np.array([1.0, -2.0])}
    G = {"w": np.array([0.5, -4.0])}
    st = {}
    for t in range(3):
        mlp.adam_step(P, G, st, lr=0.1, eps=0.0)
    np.testing.assert_allclose(P["w"], [1.0 - 0.3, -2.0 + 0.3], atol=1e-12)


def _small(seed=1, n=3, p=2):
    mesh = synth.hex_lattice(n, 0.1, seed=seed)
    ref = OracleProblem(mesh, p)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=seed + 1)
    kbar, feats = mlp.element_features(kappa, p + 2)
    nd = (p + 1) ** 3
    P = synth.mlp_init(16, 16, 16, seed=seed + 2, zero_last=False)
    V = np.random.default_rng(seed + 3).normal(size=(nd, 16)) / 4.0
    return ref, feats, P, V


def test_zero_basis_is_jacobi():
    ref, feats, P, V = _small()
    r = np.random.default_rng(4).normal(size=ref.space.ndofs)
    d = ref.Kc.diagonal()
    z, _ = mlp.precondition(P, 0.0 * V, r, d, ref.space.elem_dofs, ref.space.boundary, feats, 16)
    want = r / d
    want[ref.space.boundary] = 0.0
    np.testing.assert_allclose(z, want, atol=1e-15)


def test_preconditioner_is_symmetric_with_psd_correction():
    """Brute force: the matrix of r -> z(r) on the free dofs."""
    ref, feats, P, V = _small(seed=5, n=2)
    d = ref.Kc.diagonal()
    free = np.flatnonzero(~ref.space.boundary)
    M = np.empty((free.size, free.size))
    for j, g in enumerate(free):
        r = np.zeros(ref.space.ndofs)
        r[g] = 1.0
        z, _ = mlp.precondition(P, V, r, d, ref.space.elem_dofs, ref.space.boundary, feats, 16)
        M[:, j] = z[free]
    np.testing.assert_allclose(M, M.T, atol=1e-12 * np.abs(M).max())
    corr = M - np.diag(1.0 / d[free])
    ev = np.linalg.eigvalsh(0.5 * (corr + corr.T))
    assert ev.min() >= -1e-12 * ev.max() and ev.max() > 0
    # the correction has rank at most K per element
    assert np.linalg.matrix_rank(corr, tol=1e-10 * ev.max()) <= 16 * ref.space.elem_dofs.shape[0]


def test_preconditioner_scales_with_the_operator():
    """Scaling A by alpha scales z by 1/alpha (dbar and diag scale together); the
    log-ratio features do not change when the coefficient is scaled."""
    ref, feats, P, V = _small(seed=7)
    d = ref.Kc.diagonal()
    r = np.random.default_rng(8).normal(size=ref.space.ndofs)
    z1, _ = mlp.precondition(P, V, r, d, ref.space.elem_dofs, ref.space.boundary, feats, 16)
    z2, _ = mlp.precondition(P, V, r, 250.0 * d, ref.space.elem_dofs, ref.space.boundary, feats, 16)
    np.testing.assert_allclose(250.0 * z2, z1, rtol=1e-13, atol=1e-15)
    kappa = synth.lognormal_iid(4, 3, 1.0, seed=9)
    np.testing.assert_allclose(mlp.element_features(37.0 * kappa, 3)[1],
                               mlp.element_features(kappa, 3)[1], atol=1e-13)


def test_diag_mean_closed_form():
    ed = np.array([[0, 1, 2, 3], [2, 3, 4, 5], [4, 5, 4, 5]])
    bd = np.array([True, False, False, False, True, True])
    d = np.array([10.0, 1.0, 2.0, 3.0, 20.0, 30.0])
    np.testing.assert_allclose(mlp.diag_mean(d, ed, bd), [2.0, 2.5, 1.0])


def test_element_features_closed_form():
    kappa = np.ones((2, 27))
    kappa[1, :] = 5.0
    kbar, f = mlp.element_features(kappa, 3)
    np.testing.assert_allclose(kbar, [1.0, 5.0])
    np.testing.assert_allclose(f, 0.0, atol=1e-15)
    # a coefficient depending on x only: octants with x-high all see the same ratio
    q = np.arange(3)
    kx = np.broadcast_to(np.exp(q)[None, None, :], (3, 3, 3)).reshape(1, 27)
    kbar, f = mlp.element_features(kx, 3)
    lo, hi = 1.0, np.mean(np.exp([1.0, 2.0]))
    np.testing.assert_allclose(f[0, 0], np.log(lo / kbar[0]))
    np.testing.assert_allclose(f[0, 1], np.log(hi / kbar[0]))
    assert np.allclose(f[0, ::2], f[0, 0]) and np.allclose(f[0, 1::2], f[0, 1])


def test_loss_gradient_finite_differences():
    ref, feats, P, V = _small(seed=3, n=2)
    rng = np.random.default_rng(7)
    for k in P:
        P[k] = P[k] + 0.1 * rng.normal(size=P[k].shape)   # no dead units at zero bias
    e = rng.normal(size=ref.space.ndofs)
    e[ref.space.boundary] = 0
    A = ref.Kc
    r = A @ e
    d = A.diagonal()
    args = (A, r, e, d, ref.space.elem_dofs, ref.space.boundary, feats, 16)
    L, G = mlp.loss_and_grads(P, V, *args)
    h = 1e-6
    params = dict(P, V=V)
    for k in ("W1", "W3", "b2", "b3", "V"):
        flat = params[k].ravel()
        for idx in rng.choice(flat.size, size=4, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            Lp, _ = mlp.loss_and_grads(P, V, *args)
            flat[idx] = old - h
            Lm, _ = mlp.loss_and_grads(P, V, *args)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - G[k].ravel()[idx]) <= 1e-5 * max(1e-3, abs(fd)), (k, idx, fd)


def test_fcg_with_linear_preconditioner_equals_pcg():
    mesh = synth.hex_lattice(4, 0.1, seed=2)
    ref = OracleProblem(mesh, 2)
    b = ref.load(synth.sine_source)
    d = ref.Kc.diagonal()
    x, k, hist = mlp.fcg(ref.Kc, b, lambda r: r / d, tol=1e-10)
    r = oracle.pcg(ref.Kc, b, d, tol=1e-10)
    assert abs(k - r["iters"]) <= 1
    np.testing.assert_allclose(hist[:10], r["history"][:10], rtol=1e-6)
    xd = spla.spsolve(ref.Kc.tocsc(), b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8
