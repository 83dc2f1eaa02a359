"""Multigrid in the polynomial order (p-multigrid) as a preconditioner (oracle; test
infrastructure only).

"Scalable Linear Solvers": a partially assembled operator has no matrix entries, so
its preconditioners must be matrix-free too; the paper names multigrid over the
polynomial order among them without fixing an algorithm.  The definitions below are
this project's own, and the GPU library follows the same ones step for step:

* Levels l = 0..L-1: H1 spaces of orders p_0 >= p_1 >= ... >= p_{L-1} on one mesh.
  A_l is the constrained diffusion matrix of order p_l with q1d = p_l + 2.  Levels
  below the finest use the per-element mean of the finest coefficient (arithmetic,
  geometric or harmonic; :func:`element_mean`) at every quadrature point.
* Prolongation from level l+1 to level l: interpolation, i.e. the coarse finite
  element function evaluated at every fine node, P[i, j] = phi^c_j(x_i).  On each
  element this is the coarse tensor basis evaluated at the fine Gauss-Lobatto nodes
  (here evaluated directly in 3D, not factorised).  Used on free dofs only: rows of
  essential fine dofs and columns of essential coarse dofs are zero.  Restriction is
  its transpose.
* Smoother: Chebyshev iteration with the Jacobi preconditioner D = diag(A_l) on the
  eigenvalue interval [lo * lmax, hi * lmax] of D^-1 A_l (Saad, "Iterative Methods
  for Sparse Linear Systems", the Chebyshev acceleration algorithm of ch. 12), with
  lmax from the power iteration of :func:`power_lmax`.
* V-cycle: m smoothing steps from a zero guess, residual, restriction, recursion,
  prolongation added to the iterate, m smoothing steps.  Coarsest level: a fixed
  number of Jacobi-PCG iterations from zero (a fixed but nonlinear map, hence the
  flexible CG outside), or an exact solve.

* Levels in the mesh size (h-multigrid, the paper names h- and p-multigrid together):
  a mesh refined uniformly (:func:`refine`: every hexahedron split into 8 children that
  cover the octants of its reference cube, axes kept) holds the coarse mesh's space,
  because each child's map is the parent's map restricted to the octant.  The
  prolongation from a coarse level on the parent mesh to a fine level on the refined
  mesh is again interpolation: the coarse function on the parent evaluated at the
  child's nodes, i.e. the coarse basis at the parent reference points (o + xhat) / 2
  of octant o (:func:`h_interpolation`).  A level's coefficient is the mean of the
  finest coefficient over every finest point inside the level's element
  (:func:`level_coefficient`); children are numbered 8 e + o, so those points are
  contiguous.  :func:`build_hp_levels` mixes both kinds of step.

Pins (tests/test_oracle_pmg.py): interpolation reproduces functions of the coarse
space exactly and sums to one per row; P^T K_f P equals the coarse stiffness (and
mass) matrix on affine meshes with a constant coefficient (both are the exact
Galerkin matrices there); Chebyshev error equals the scaled Chebyshev polynomial
per eigenvalue; the power iteration converges to the largest eigenvalue from below;
a V-cycle whose coarse level is the fine space solved exactly returns A^-1 b; the
cycle with an exact coarse solve is symmetric positive definite; closed-form means.
Refinement (tests/test_oracle_hmg.py): child vertices and quadrature points are the
parent's map at the octant's points, volumes add up, the refined mesh is conforming
(its H1 space has the dof count of the lattice twice as fine); h-interpolation
reproduces linear functions and, on affine meshes, P^T A_f P is the coarse matrix.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .basis import tensor_basis, tensor_points
from .geometry import map_points
from .quadrature import gauss_lobatto
from .solvers import pcg
from .space import H1Space


def element_mean(coeff, kind="arithmetic"):
    """Per-element mean [E] of a coefficient given per quadrature point [E, Q^3]."""
    c = np.asarray(coeff, dtype=np.float64)
    if kind == "arithmetic":
        return c.mean(axis=1)
    if kind == "geometric":
        return np.exp(np.log(c).mean(axis=1))
    if kind == "harmonic":
        return 1.0 / (1.0 / c).mean(axis=1)
    raise ValueError(kind)


def interpolation(mesh, pc, pf, free_only=True):
    """CSR prolongation [ndof_f, ndof_c] from order pc to order pf on ``mesh``."""
    Sc, Sf = H1Space(mesh, pc), H1Space(mesh, pf)
    PE, _ = tensor_basis(gauss_lobatto(pc + 1), tensor_points(gauss_lobatto(pf + 1)))
    E = Sc.elem_dofs.shape[0]
    rows = np.repeat(Sf.elem_dofs, PE.shape[1], axis=1).ravel()
    cols = np.tile(Sc.elem_dofs, (1, PE.shape[0])).ravel()
    vals = np.broadcast_to(PE.ravel()[None, :], (E, PE.size)).ravel()
    # every element holding both dofs gives the same entry: keep one of them
    key = rows.astype(np.int64) * Sc.ndofs + cols
    _, first = np.unique(key, return_index=True)
    P = sp.csr_matrix((vals[first], (rows[first], cols[first])), shape=(Sf.ndofs, Sc.ndofs))
    if free_only:
        P = sp.diags((~Sf.boundary).astype(float)) @ P @ sp.diags((~Sc.boundary).astype(float))
    return P.tocsr()


def power_lmax(A, diag, v0, iters):
    """Largest eigenvalue estimate of D^-1 A by power iteration, D = diag(diag).

    v_0 = v0 normalised in the D-norm; for k = 1..iters: w = A v_{k-1},
    lambda_k = v_{k-1} . w, v_k = D^-1 w / ||D^-1 w||_D.  Returns lambda_iters.
    """
    d = np.asarray(diag, dtype=np.float64)
    v = np.asarray(v0, dtype=np.float64) / np.sqrt(np.sum(d * v0 * v0))
    lam = 0.0
    for _ in range(iters):
        w = A @ v
        lam = v @ w
        u = w / d
        v = u / np.sqrt(np.sum(d * u * u))
    return lam


def chebyshev(A, diag, b, x, lmax, degree, lo=0.3, hi=1.1):
    """``degree`` steps of Jacobi-preconditioned Chebyshev iteration on A x = b.

    Eigenvalue interval [lo lmax, hi lmax]; theta and delta its centre and half
    width, sigma = theta / delta.  r_0 = b - A x_0, rho_0 = 1/sigma,
    d_0 = D^-1 r_0 / theta; then x_{k+1} = x_k + d_k, r_{k+1} = r_k - A d_k,
    rho_{k+1} = 1 / (2 sigma - rho_k), d_{k+1} = rho_{k+1} rho_k d_k
    + (2 rho_{k+1} / delta) D^-1 r_{k+1}.  x = None means x_0 = 0.
    """
    theta = 0.5 * (hi + lo) * lmax
    delta = 0.5 * (hi - lo) * lmax
    sigma = theta / delta
    x = np.zeros_like(b) if x is None else np.array(x, dtype=np.float64)
    r = b - A @ x
    rho = 1.0 / sigma
    d = r / (theta * diag)
    for k in range(degree):
        x = x + d
        if k == degree - 1:
            break
        r = r - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (r / diag)
        rho = rho_new
    return x


def vcycle(levels, b, level=0, degree=2, lo=0.3, hi=1.1, coarse_iters=None):
    """One V-cycle from a zero guess.  ``levels[l]``: dict with A, diag, lmax, and
    (l < L-1) P, the prolongation from level l+1 to level l.
    coarse_iters=None solves the coarsest level exactly."""
    L = levels[level]
    if level == len(levels) - 1:
        if coarse_iters is None:
            return spla.spsolve(L["A"].tocsc(), b)
        return pcg(L["A"], b, L["diag"], tol=0.0, maxiter=coarse_iters)["x"]
    x = chebyshev(L["A"], L["diag"], b, None, L["lmax"], degree, lo, hi)
    r = b - L["A"] @ x
    bc = L["P"].T @ r
    xc = vcycle(levels, bc, level + 1, degree, lo, hi, coarse_iters)
    x = x + L["P"] @ xc
    return chebyshev(L["A"], L["diag"], b, x, L["lmax"], degree, lo, hi)


def default_orders(p):
    """p, then halved (rounding down) until 1."""
    out = [p]
    while out[-1] > 1:
        out.append(max(1, out[-1] // 2))
    return out


def build_levels(mesh, orders, coeff=None, mean="arithmetic", starts=None, power_iters=20):
    """Levels for :func:`vcycle`: constrained stiffness matrices of each order (the
    coarse ones with the element mean of ``coeff``), their diagonals, lmax by
    :func:`power_lmax` from ``starts[l]`` (one start vector per level, in the
    level's oracle dof order), and the prolongations between consecutive orders.
    Also returns the spaces (for dof coordinates)."""
    from .forms import assemble, constrain, element_stiffness
    levels, spaces = [], []
    for l, p in enumerate(orders):
        S = H1Space(mesh, p)
        q = p + 2
        if coeff is None:
            c = None
        elif l == 0:
            c = coeff
        else:
            c = np.repeat(element_mean(coeff, mean)[:, None], q ** 3, axis=1)
        K = assemble(S, element_stiffness(mesh, p, q, c))
        Kc, _ = constrain(K, np.zeros(S.ndofs), S.boundary)
        d = Kc.diagonal()
        lv = {"A": Kc, "diag": d, "p": p}
        if starts is not None:
            lv["lmax"] = power_lmax(Kc, d, np.where(S.boundary, 0.0, starts[l]), power_iters)
        levels.append(lv)
        spaces.append(S)
    for l in range(len(orders) - 1):
        levels[l]["P"] = interpolation(mesh, orders[l + 1], orders[l])
    return levels, spaces


# reference corner of each slot of the usual hexahedron vertex order
_SLOT_CORNER = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                         [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]])


def _octant(o):
    return np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1], dtype=np.float64)


def refine(mesh):
    """Uniform refinement of a hexahedral mesh dict.

    Child 8 e + o (o = ox + 2 oy + 4 oz) of element e covers the parent's reference
    box [o/2, (o+1)/2] with its axes along the parent's.  The fine vertices are the
    nodes of the parent mesh's order-2 H1 space (corners, edge midpoints, face and cell
    centres of every reference cube), identified topologically by that space and placed
    by the parent's map; a quadratic geometry gives each child the parent's map at its
    27 nodes, so in both cases the child's map is the parent's on the octant."""
    S2 = H1Space(mesh, 2)
    X2, _ = map_points(mesh, tensor_points(np.array([0.0, 0.5, 1.0])))     # [E, 27, 3]
    E = S2.elem_dofs.shape[0]
    verts = np.empty((S2.ndofs, 3))
    verts[S2.elem_dofs.ravel()] = X2.reshape(-1, 3)
    hexes = np.empty((E, 8, 8), dtype=np.int64)
    for o in range(8):
        off = _octant(o).astype(np.int64)
        for s, c in enumerate(_SLOT_CORNER):
            i, j, k = off + c
            hexes[:, o, s] = S2.elem_dofs[:, i + 3 * j + 9 * k]
    out = {"vertices": verts, "hex": hexes.reshape(E * 8, 8)}
    if mesh.get("geom_order", 1) == 2 and mesh.get("geom_nodes") is not None:
        g = np.empty((E, 8, 27, 3))
        ref = tensor_points(np.array([0.0, 0.5, 1.0]))
        for o in range(8):
            g[:, o], _ = map_points(mesh, (_octant(o) + ref) / 2.0)
        out["geom_order"] = 2
        out["geom_nodes"] = g.reshape(E * 8, 27, 3)
    return out


def h_interpolation(coarse_mesh, fine_mesh, pc, pf, free_only=True):
    """CSR prolongation [ndof_f, ndof_c] from order pc on ``coarse_mesh`` to order pf
    on ``fine_mesh = refine(coarse_mesh)``: P[i, j] = phi^c_j at fine node i, the
    coarse basis of the parent evaluated at (o + xhat_i) / 2 for a child in octant o."""
    Sc, Sf = H1Space(coarse_mesh, pc), H1Space(fine_mesh, pf)
    Ec = Sc.elem_dofs.shape[0]
    assert Sf.elem_dofs.shape[0] == 8 * Ec, "fine mesh is not a refinement of the coarse one"
    xf = tensor_points(gauss_lobatto(pf + 1))
    rows, cols, vals = [], [], []
    for o in range(8):
        PE, _ = tensor_basis(gauss_lobatto(pc + 1), (_octant(o) + xf) / 2.0)
        child = 8 * np.arange(Ec) + o
        rows.append(np.repeat(Sf.elem_dofs[child], PE.shape[1], axis=1).ravel())
        cols.append(np.tile(Sc.elem_dofs, (1, PE.shape[0])).ravel())
        vals.append(np.broadcast_to(PE.ravel()[None, :], (Ec, PE.size)).ravel())
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    key = rows.astype(np.int64) * Sc.ndofs + cols
    _, first = np.unique(key, return_index=True)
    P = sp.csr_matrix((vals[first], (rows[first], cols[first])), shape=(Sf.ndofs, Sc.ndofs))
    if free_only:
        P = sp.diags((~Sf.boundary).astype(float)) @ P @ sp.diags((~Sc.boundary).astype(float))
    return P.tocsr()


def level_coefficient(coeff, n_elements, q, kind="arithmetic"):
    """Coefficient [n_elements, q^3] of a coarse level: the mean of the finest
    coefficient [E_0, Q^3] over the finest points inside each of the level's elements
    (a contiguous block of E_0 / n_elements finest elements), at every point."""
    c = np.asarray(coeff, dtype=np.float64).reshape(n_elements, -1)
    return np.repeat(element_mean(c, kind)[:, None], q ** 3, axis=1)


def build_hp_levels(meshes, plan, coeff=None, mean="arithmetic", starts=None, power_iters=20):
    """Levels for :func:`vcycle` in mesh size and order.  ``meshes[0]`` is the finest
    mesh and ``meshes[k] = refine(meshes[k+1])``; ``plan`` lists (mesh index, order)
    per level, finest first, each step either lowering the order on one mesh or moving
    to the parent mesh (order not raised).  Same conventions as :func:`build_levels`."""
    from .forms import assemble, constrain, element_stiffness
    levels, spaces = [], []
    for l, (m, p) in enumerate(plan):
        mesh = meshes[m]
        S = H1Space(mesh, p)
        q = p + 2
        if coeff is None:
            c = None
        elif l == 0:
            c = coeff
        else:
            c = level_coefficient(coeff, S.elem_dofs.shape[0], q, mean)
        K = assemble(S, element_stiffness(mesh, p, q, c))
        Kc, _ = constrain(K, np.zeros(S.ndofs), S.boundary)
        d = Kc.diagonal()
        lv = {"A": Kc, "diag": d, "p": p, "mesh": m}
        if starts is not None:
            lv["lmax"] = power_lmax(Kc, d, np.where(S.boundary, 0.0, starts[l]), power_iters)
        levels.append(lv)
        spaces.append(S)
    for l in range(len(plan) - 1):
        (mf, pf), (mc, pc) = plan[l], plan[l + 1]
        if mc == mf:
            levels[l]["P"] = interpolation(meshes[mf], pc, pf)
        elif mc == mf + 1:
            levels[l]["P"] = h_interpolation(meshes[mc], meshes[mf], pc, pf)
        else:
            raise ValueError("a level step moves to the same mesh or its parent")
    return levels, spaces
