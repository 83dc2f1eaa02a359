"""Element matrices, load vectors, global assembly and essential BCs (oracle; test infrastructure only).

Definitions followed:

* Diffusion (stiffness) entries A_ij = int grad phi_j . grad phi_i, with a
  coefficient kappa inside the integral -- "Finite Element Abstractions",
  eq. (abstract forms) and the matrix definition before eq. (linear system).
  Mapped to the reference element with quadrature (the same change of
  variables as the mass-matrix equations of "High-Order Partial Assembly"):
      K_E[i, j] = sum_k alpha_k kappa_k det J_k (J_k^{-T} ghat_i) . (J_k^{-T} ghat_j).
  The quadrature-point factor alpha kappa det J J^{-1} J^{-T} is computed with a
  matrix inverse (numpy.linalg.inv), not with the adjugate form of the paper's
  2D setup listing ("GPU Acceleration"), which is what the test pins it against.
* Mass M_E = B^t D_E B, (D_E)_kk = alpha_k det J(xhat_k) rho(Phi(xhat_k)) --
  "High-Order Partial Assembly", mass-matrix equations.
* Load b_i = int f phi_i -- eq. (abstract forms), the b_i definition.
* Convection C_E[i, j] = sum_k alpha_k det J_k phi_i (beta . J_k^{-T} ghat_j), the
  form int (beta . grad u) v with J^{-1} again from numpy.linalg.inv.
* Gradient G_E[c, i, j] = sum_k alpha_k kappa_k det J_k phi_i (J_k^{-T} ghat_j)_c, the
  mixed form (grad u, v) with v vector-valued in the same space.
* Divergence V_E[c, i, j] = sum_k alpha_k kappa_k det J_k phi_i (d phi_j / d x_c)(x_k),
  the mixed form (div u, q) with u vector-valued; the physical gradient here comes
  from solving J^T g = ghat (numpy.linalg.solve), not from an inverse.
* Linear elasticity K_E[c, i, d, j] = sum_k alpha_k det J_k [lambda d_c phi_i d_d phi_j +
  mu (delta_cd grad phi_i . grad phi_j + d_d phi_i d_c phi_j)], the bilinear form
  int lambda div u div v + 2 mu eps(u):eps(v) on the vector H1 space (component-major).
* Global operator A = sum_E G_E^t A_E G_E (dense element matrices scattered into
  a sparse matrix; "Operator Decomposition" with P = identity).
* Essential BC: the "further modifications" of FormLinearSystem ("Finite Element
  Linear Systems") are not spelled out; the reading used is symmetric elimination:
  zero the boundary rows and columns, unit diagonal, b_G = g, b_I -= A_IG g.

Pins (tests/test_oracle_forms.py): closed-form 1D element matrices on affine
cubes, volume = 1^T M 1, K 1 = 0, SPD with nullity 1 before BC, the paper's 2D
setup formula, linear patch test, O(h^{p+1}) L2 convergence; divergence of linear
vector fields, integration by parts against the gradient matrices, affine closed form;
elasticity rigid-body null space, linear patch test, lambda and mu parts against the
gradient and diffusion matrices, affine closed form.
"""
import numpy as np
import scipy.sparse as sp

from .basis import tensor_basis, tensor_points, tensor_weights
from .geometry import map_points
from .quadrature import gauss_legendre, gauss_lobatto


def quadrature_points(q1d):
    """Tensor Gauss-Legendre points [Q^3, 3] and weights [Q^3] on [0,1]^3 (x fastest)."""
    x, w = gauss_legendre(q1d)
    return tensor_points(x), tensor_weights(w)


def qpoint_diffusion_operator(J, weight, coeff=1.0):
    """alpha * coeff * det J * J^{-1} J^{-T} for Jacobians J[..., d, d] (any d)."""
    J = np.asarray(J, dtype=np.float64)
    Jinv = np.linalg.inv(J)
    det = np.linalg.det(J)
    scale = np.asarray(weight) * np.asarray(coeff) * det
    return scale[..., None, None] * np.einsum("...ab,...cb->...ac", Jinv, Jinv)


def _jacobians(mesh, q1d):
    pts, w = quadrature_points(q1d)
    x, J = map_points(mesh, pts)
    det = np.linalg.det(J)
    if np.any(det <= 0.0):
        bad = int(np.nonzero((det <= 0.0).any(axis=1))[0][0])
        raise ValueError(f"non-positive Jacobian determinant in element {bad}")
    return pts, w, x, J, det


def _chunks(E, per_elem_bytes, budget=256 << 20):
    step = max(1, int(budget // max(per_elem_bytes, 1)))
    for a in range(0, E, step):
        yield slice(a, min(E, a + step))


def element_stiffness(mesh, p, q1d, coeff=None):
    """Dense element diffusion matrices [E, D^3, D^3]; coeff is None, scalar or [E, Q^3].

    K_E = sum_q ghat(q)^T Dq ghat(q), evaluated as one matrix product per element:
    with Ghat = [ghat_1; ghat_2; ghat_3] of shape [3 Q^3, D^3] and H = Dq applied
    pointwise to Ghat, K_E = Ghat^T H.
    """
    pts, w, _, J, _ = _jacobians(mesh, q1d)
    _, grad = tensor_basis(gauss_lobatto(p + 1), pts)                  # [3, Q^3, D^3]
    c = 1.0 if coeff is None else coeff
    Dq = qpoint_diffusion_operator(J, w[None, :], c)                   # [E, Q^3, 3, 3]
    E, nq, nd = J.shape[0], grad.shape[1], grad.shape[2]
    gflat = grad.reshape(3 * nq, nd)
    out = np.empty((E, nd, nd))
    for sl in _chunks(E, 8 * 3 * nq * nd):
        H = np.einsum("eqab,bqj->eaqj", Dq[sl], grad).reshape(-1, 3 * nq, nd)
        out[sl] = np.matmul(gflat.T[None], H)
    return out


def element_mass(mesh, p, q1d, coeff=None):
    """Dense element mass matrices [E, D^3, D^3]: M_E = B^t diag(alpha det J rho) B."""
    pts, w, _, _, det = _jacobians(mesh, q1d)
    val, _ = tensor_basis(gauss_lobatto(p + 1), pts)                   # [Q^3, D^3]
    c = 1.0 if coeff is None else coeff
    d = w[None, :] * det * c
    E, nd = det.shape[0], val.shape[1]
    out = np.empty((E, nd, nd))
    for sl in _chunks(E, 8 * val.size):
        out[sl] = np.matmul(val.T[None], d[sl][:, :, None] * val[None])
    return out


def element_load(mesh, p, q1d, f):
    """Element load vectors [E, D^3] for b_i = int f phi_i.

    ``f`` is a callable on physical points [E, Q^3, 3] or an array [E, Q^3].
    """
    pts, w, x, _, det = _jacobians(mesh, q1d)
    val, _ = tensor_basis(gauss_lobatto(p + 1), pts)
    fq = f(x) if callable(f) else np.asarray(f)
    return np.einsum("qi,eq->ei", val, w[None, :] * det * fq)


def element_convection(mesh, p, q1d, velocity):
    """Dense element convection matrices [E, D^3, D^3] for a(u, v) = int (beta . grad u) v.

    C_E[i, j] = sum_k alpha_k det J_k phi_i(xhat_k) beta_k . (J_k^{-T} ghat_j(xhat_k))
    ("Finite Element Abstractions", the bilinear form; the convection integrator is
    one of the partially assembled integrators listed in "GPU Acceleration").
    ``velocity`` is a callable on physical points [E, Q^3, 3], a 3-vector, or an
    array [E, Q^3, 3].
    """
    pts, w, x, J, det = _jacobians(mesh, q1d)
    val, grad = tensor_basis(gauss_lobatto(p + 1), pts)               # [Q^3, D^3], [3, Q^3, D^3]
    if callable(velocity):
        beta = velocity(x)
    else:
        beta = np.broadcast_to(np.asarray(velocity, dtype=np.float64), x.shape)
    Jinv = np.linalg.inv(J)                                            # [E, Q^3, 3, 3]
    # beta . J^{-T} g = (J^{-1} beta) . g
    c = np.einsum("eqba,eqa->eqb", Jinv, beta) * (w[None, :] * det)[..., None]   # [E, Q^3, 3]
    dphi = np.einsum("eqb,bqj->eqj", c, grad)                          # [E, Q^3, D^3]
    return np.einsum("qi,eqj->eij", val, dphi)


def element_gradient(mesh, p, q1d, coeff=None):
    """Dense element gradient matrices [E, 3, D^3, D^3] of the mixed form
    (grad u, v) with u and each component of v in the same H1 space:

        G_E[c, i, j] = sum_k alpha_k kappa_k det J_k phi_i(xhat_k) (J_k^{-T} ghat_j)_c,

    the gradient integrator among the paper's partially assembled kernels ("GPU
    Acceleration"); coeff None, scalar or [E, Q^3].
    """
    pts, w, _, J, det = _jacobians(mesh, q1d)
    val, grad = tensor_basis(gauss_lobatto(p + 1), pts)               # [Q^3, D^3], [3, Q^3, D^3]
    c = 1.0 if coeff is None else np.asarray(coeff)
    Jinv = np.linalg.inv(J)                                            # [E, Q^3, 3, 3]
    scale = (w[None, :] * det) * c                                     # [E, Q^3]
    # (J^{-T} g)_c = sum_b Jinv[b, c] g_b
    phys = np.einsum("eqbc,bqj->ecqj", Jinv, grad)                     # [E, 3, Q^3, D^3]
    return np.einsum("qi,eq,ecqj->ecij", val, scale, phys)


def element_divergence(mesh, p, q1d, coeff=None):
    """Dense element divergence matrices [E, 3, D^3, D^3] of the mixed form
    (div u, q) with each component of u and the scalar q in the same H1 space (the
    divergence integrator among the paper's partially assembled kernels, "GPU
    Acceleration"):

        V_E[c, i, j] = sum_k alpha_k kappa_k det J_k phi_i(xhat_k) (d phi_j / d x_c)(x_k),

    so that (V u)_i = sum_c sum_j V[c, i, j] u_c[j] is the load of div u against
    phi_i.  The physical gradient is obtained by solving J^T g = ghat at each point;
    coeff None, scalar or [E, Q^3].
    """
    pts, w, _, J, det = _jacobians(mesh, q1d)
    val, grad = tensor_basis(gauss_lobatto(p + 1), pts)               # [Q^3, D^3], [3, Q^3, D^3]
    c = 1.0 if coeff is None else np.asarray(coeff)
    E, nq = det.shape
    Jt = np.broadcast_to(np.swapaxes(J, -1, -2)[:, :, None], (E, nq, grad.shape[2], 3, 3))
    rhs = np.broadcast_to(np.moveaxis(grad, 0, -1)[None], (E, nq, grad.shape[2], 3))
    phys = np.linalg.solve(Jt, rhs[..., None])[..., 0]                # [E, Q^3, D^3, 3]
    scale = (w[None, :] * det) * c                                     # [E, Q^3]
    return np.einsum("qi,eq,eqjc->ecij", val, scale, phys)


def element_elasticity(mesh, p, q1d, lam, mu):
    """Dense element matrices [E, 3, D^3, 3, D^3] of isotropic linear elasticity on the
    vector H1 space (each displacement component in the scalar space):

        a(u, v) = int lambda (div u)(div v) + 2 mu eps(u) : eps(v),  eps(u) = (grad u + grad u^T)/2,

    which for u = phi_j e_d, v = phi_i e_c gives

        K_E[c, i, d, j] = sum_k alpha_k det J_k [ lambda_k d_c phi_i d_d phi_j
                          + mu_k (delta_cd grad phi_i . grad phi_j + d_d phi_i d_c phi_j) ],

    d_c the physical derivative (J^{-T} ghat)_c; lam and mu scalars or [E, Q^3].
    """
    pts, w, _, J, det = _jacobians(mesh, q1d)
    _, grad = tensor_basis(gauss_lobatto(p + 1), pts)                 # [3, Q^3, D^3]
    Jinv = np.linalg.inv(J)                                            # [E, Q^3, 3, 3]
    phys = np.einsum("eqbc,bqj->eqjc", Jinv, grad)                     # [E, Q^3, D^3, 3]
    wd = w[None, :] * det
    lw = wd * np.asarray(lam)                                          # [E, Q^3]
    mw = wd * np.asarray(mu)
    E, nq, nd, _ = phys.shape
    Pm = phys.reshape(E, nq, nd * 3)                                   # column (j, c)

    def gram(wq):
        # [e, i, a, j, b] = sum_q wq d_a phi_i d_b phi_j, as one matrix product per element
        return np.matmul(np.swapaxes(Pm * wq[:, :, None], 1, 2), Pm).reshape(E, nd, 3, nd, 3)

    L, M = gram(lw), gram(mw)
    K = L.transpose(0, 2, 1, 4, 3) + M.transpose(0, 4, 1, 2, 3)       # lambda and d_d phi_i d_c phi_j
    lap = np.einsum("eiaja->eij", M)                                   # mu grad phi_i . grad phi_j
    for c in range(3):
        K[:, c, :, c, :] += lap
    return K


def vector_space(space):
    """The three-component space of `space`, component-major global index c * N + i,
    as the (elem_dofs, ndofs, boundary) triple that :func:`assemble` and
    :func:`constrain` take."""
    from types import SimpleNamespace
    n = space.ndofs
    ed = np.concatenate([space.elem_dofs + c * n for c in range(3)], axis=1)
    return SimpleNamespace(elem_dofs=ed, ndofs=3 * n, boundary=np.tile(space.boundary, 3))


def assemble(space, elmats):
    """Global CSR sum_E G_E^t A_E G_E (duplicates summed)."""
    E, nd, _ = elmats.shape
    rows = np.repeat(space.elem_dofs, nd, axis=1).ravel()
    cols = np.tile(space.elem_dofs, (1, nd)).ravel()
    A = sp.coo_matrix((elmats.ravel(), (rows, cols)), shape=(space.ndofs, space.ndofs))
    return A.tocsr()


def assemble_vector(space, elvecs):
    """Global vector sum_E G_E^t v_E."""
    return np.bincount(space.elem_dofs.ravel(), weights=np.asarray(elvecs).ravel(),
                       minlength=space.ndofs)


def constrain(A, b, boundary_mask, g=None):
    """Symmetric elimination of essential dofs with a unit diagonal.

    Returns (A_c, b_c) with A_c[G, :] = A_c[:, G] = 0 except A_c[G, G] = I,
    b_c[G] = g and b_c[I] = b[I] - A[I, G] g.
    """
    n = A.shape[0]
    bmask = np.asarray(boundary_mask, dtype=bool)
    gvec = np.zeros(n) if g is None else np.asarray(g, dtype=np.float64)
    keep = sp.diags((~bmask).astype(np.float64))
    Ac = (keep @ A @ keep + sp.diags(bmask.astype(np.float64))).tocsr()
    bc = np.asarray(b, dtype=np.float64) - A @ np.where(bmask, gvec, 0.0)
    bc[bmask] = gvec[bmask]
    return Ac, bc
