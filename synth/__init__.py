"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only *generates inputs*: hexahedral and quadrilateral lattice meshes
(optionally jittered, warped or with rotated element vertex lists), coefficient fields
and right-hand-side vectors.  It holds none of the finite element arithmetic (no basis, no quadrature
operator, no assembly); both the CPU oracle and the HIP library consume its arrays.

Conventions fixed here and used by both sides:

* Hex connectivity uses the common vertex order of a hexahedron: bottom face
  (0,0,0) (1,0,0) (1,1,0) (0,1,0), then the top face in the same order.
* Quadrature-point arrays are indexed ``[element][qx + Q*(qy + Q*qz)]``.
* The domain is the unit cube; jitter moves interior vertices only, so the
  boundary and the volume stay exact.
"""
from __future__ import annotations

import numpy as np

# Corner coordinates of the reference cube in hexahedron vertex order.
HEX_CORNERS = np.array(
    [[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
     [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)


def _rotation_matrices() -> list[np.ndarray]:
    """The 24 proper rotations of the cube as signed permutation matrices."""
    import itertools
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            m = np.zeros((3, 3), dtype=np.int64)
            for r, (c, s) in enumerate(zip(perm, signs)):
                m[r, c] = s
            if round(np.linalg.det(m)) == 1:
                mats.append(m)
    assert len(mats) == 24
    return mats


def _corner_permutations() -> np.ndarray:
    """perm[r][s] = which old vertex slot becomes new slot s under rotation r."""
    lookup = {tuple(c): i for i, c in enumerate(HEX_CORNERS)}
    out = []
    for m in _rotation_matrices():
        centred = 2 * HEX_CORNERS - 1              # corners at +-1
        rotated = (centred @ m.T + 1) // 2          # back to {0,1}
        out.append([lookup[tuple(c)] for c in rotated])
    return np.array(out, dtype=np.int64)


CUBE_ROTATIONS = _corner_permutations()  # [24, 8]


def hex_lattice(n, jitter: float = 0.0, seed: int = 0,
                rotate_seed: int | None = None) -> dict:
    """Unit-cube lattice of nx*ny*nz hexahedra (n is an int or a 3-tuple).

    Interior vertices are displaced by ``jitter * h * u`` with ``u`` uniform in the
    unit ball (h = 1/max(n)), using ``numpy.random.default_rng(seed)``.  With
    ``rotate_seed`` every element's vertex list is re-labelled by a random proper
    rotation of the cube (same geometry, different local orientation).
    Elements are numbered lexicographically (x fastest).
    """
    nx, ny, nz = (int(n),) * 3 if np.isscalar(n) else tuple(int(v) for v in n)
    mx, my, mz = nx + 1, ny + 1, nz + 1
    vz, vy, vx = np.meshgrid(np.arange(mz) / nz, np.arange(my) / ny, np.arange(mx) / nx,
                             indexing="ij")
    verts = np.stack([vx.ravel(), vy.ravel(), vz.ravel()], axis=1)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        nv = verts.shape[0]
        d = rng.normal(size=(nv, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = rng.uniform(size=(nv, 1)) ** (1.0 / 3.0)
        disp = jitter * (1.0 / max(nx, ny, nz)) * r * d
        ix = np.arange(nv)
        i0, i1, i2 = ix % mx, (ix // mx) % my, ix // (mx * my)
        interior = (i0 > 0) & (i0 < nx) & (i1 > 0) & (i1 < ny) & (i2 > 0) & (i2 < nz)
        verts[interior] += disp[interior]
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    hexes = np.empty((nx * ny * nz, 8), dtype=np.int64)
    for s, (cx, cy, cz) in enumerate(HEX_CORNERS):
        hexes[:, s] = (ex + cx) + mx * ((ey + cy) + my * (ez + cz))
    if rotate_seed is not None:
        rng = np.random.default_rng(rotate_seed)
        pick = rng.integers(0, 24, size=hexes.shape[0])
        perms = CUBE_ROTATIONS[pick]
        hexes = np.take_along_axis(hexes, perms, axis=1)
    return {"vertices": verts, "hex": hexes, "n": (nx, ny, nz), "geom_order": 1,
            "geom_nodes": None}


# Corner coordinates of the reference square in quadrilateral vertex order
# (counter-clockwise from the origin).
QUAD_CORNERS = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=np.int64)


def quad_lattice(n, jitter: float = 0.0, seed: int = 0,
                 rotate_seed: int | None = None) -> dict:
    """Unit-square lattice of nx*ny quadrilaterals (n is an int or a 2-tuple).

    Interior vertices are displaced by ``jitter * h * u`` with ``u`` uniform in the
    unit disc (h = 1/max(n)), using ``numpy.random.default_rng(seed)``.  With
    ``rotate_seed`` every element's vertex list is cyclically shifted by a random
    amount (a proper rotation of the square: same geometry, other local frame).
    Elements are numbered lexicographically (x fastest).
    """
    nx, ny = (int(n),) * 2 if np.isscalar(n) else tuple(int(v) for v in n)
    mx, my = nx + 1, ny + 1
    vy, vx = np.meshgrid(np.arange(my) / ny, np.arange(mx) / nx, indexing="ij")
    verts = np.stack([vx.ravel(), vy.ravel()], axis=1)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        nv = verts.shape[0]
        d = rng.normal(size=(nv, 2))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = np.sqrt(rng.uniform(size=(nv, 1)))
        disp = jitter * (1.0 / max(nx, ny)) * r * d
        ix = np.arange(nv)
        i0, i1 = ix % mx, ix // mx
        interior = (i0 > 0) & (i0 < nx) & (i1 > 0) & (i1 < ny)
        verts[interior] += disp[interior]
    ey, ex = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey = ex.ravel(), ey.ravel()
    quads = np.empty((nx * ny, 4), dtype=np.int64)
    for s, (cx, cy) in enumerate(QUAD_CORNERS):
        quads[:, s] = (ex + cx) + mx * (ey + cy)
    if rotate_seed is not None:
        rng = np.random.default_rng(rotate_seed)
        shift = rng.integers(0, 4, size=quads.shape[0])
        idx = (np.arange(4)[None, :] + shift[:, None]) % 4
        quads = np.take_along_axis(quads, idx, axis=1)
    return {"vertices": verts, "quad": quads, "n": (nx, ny), "geom_order": 1,
            "geom_nodes": None}


def sub_mesh(mesh: dict, elems) -> dict:
    """The mesh restricted to the listed elements (vertex array kept whole)."""
    out = dict(mesh)
    if "quad" in mesh:
        out["quad"] = mesh["quad"][elems]
        return out
    out["hex"] = mesh["hex"][elems]
    if mesh.get("geom_nodes") is not None:
        out["geom_nodes"] = mesh["geom_nodes"][elems]
    return out


def warp_sine(points: np.ndarray, amp: float) -> np.ndarray:
    """x -> x + amp * sin(2 pi x) sin(2 pi y) sin(2 pi z) * (1, 1, 1)."""
    s = np.prod(np.sin(2.0 * np.pi * points), axis=-1, keepdims=True)
    return points + amp * s


def q2_warped_lattice(n: int, amp: float = 0.05) -> dict:
    """Unit-cube lattice with quadratic (27-node) element geometry, warped.

    Geometry nodes are the lattice points at reference positions {0, 1/2, 1} per axis,
    ordered lexicographically (x fastest) per element, moved by :func:`warp_sine`.
    The warp vanishes on the boundary, so the domain stays the unit cube.
    """
    mesh = hex_lattice(n)
    h = 1.0 / n
    ez, ey, ex = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([ex.ravel(), ey.ravel(), ez.ravel()], axis=1).astype(np.float64) * h
    t = np.array([0.0, 0.5, 1.0]) * h
    gz, gy, gx = np.meshgrid(t, t, t, indexing="ij")
    offs = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)          # [27, 3]
    nodes = base[:, None, :] + offs[None, :, :]
    mesh["geom_nodes"] = warp_sine(nodes, amp)
    mesh["vertices"] = warp_sine(mesh["vertices"], amp)
    mesh["geom_order"] = 2
    return mesh


def lognormal_iid(num_elems: int, q1d: int, sigma: float = 1.0, seed: int = 0,
                  dim: int = 3) -> np.ndarray:
    """kappa[e, q] = exp(Z), Z ~ N(0, sigma^2) i.i.d. per element and quadrature point
    (q1d^dim points per element)."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.normal(size=(num_elems, q1d ** dim)))


def lattice_quadrature_points(n: int, q1d: int) -> np.ndarray:
    """Gauss-Legendre points of every element of the *undeformed* n^3 lattice.

    Returns [n^3, q1d^3, 3] in the element and point order used everywhere else.
    Used only to place coefficient fields; the solvers never read it.
    """
    xg, _ = np.polynomial.legendre.leggauss(q1d)
    xg = 0.5 * (xg + 1.0)
    qz, qy, qx = np.meshgrid(xg, xg, xg, indexing="ij")
    ref = np.stack([qx.ravel(), qy.ravel(), qz.ravel()], axis=1)
    ez, ey, ex = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([ex.ravel(), ey.ravel(), ez.ravel()], axis=1).astype(np.float64)
    return (base[:, None, :] + ref[None, :, :]) / n


def grf_lognormal(points, ell: float = 0.1, contrast: float = 1e3, seed: int = 0,
                  modes: int = 1024, device=None):
    """Lognormal field exp(s * g(x)) with g a unit-variance Gaussian field.

    g uses random Fourier features of a squared-exponential covariance with
    correlation length ``ell``; s is chosen so max/min of the field over the given
    points equals ``contrast``.  With ``device`` (a torch device) the features are
    evaluated there in float64 and a torch tensor is returned: same frequencies and
    phases, values equal to the host ones up to the rounding of cos.
    """
    rng = np.random.default_rng(seed)
    omega = rng.normal(scale=1.0 / ell, size=(modes, 3))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=modes)
    shape = np.asarray(points).shape[:-1] if device is None else tuple(points.shape[:-1])
    step = 1 << 16
    if device is None:
        flat = np.asarray(points).reshape(-1, 3)
        g = np.empty(flat.shape[0])
        for a in range(0, flat.shape[0], step):
            g[a:a + step] = np.sqrt(2.0 / modes) * np.cos(flat[a:a + step] @ omega.T + phase).sum(axis=1)
        s = np.log(contrast) / (g.max() - g.min())
        return np.exp(s * g).reshape(shape)
    import torch
    flat = torch.as_tensor(np.asarray(points) if not torch.is_tensor(points) else points,
                           dtype=torch.float64, device=device).reshape(-1, 3)
    om = torch.as_tensor(omega.T.copy(), device=device)
    ph = torch.as_tensor(phase, device=device)
    g = torch.empty(flat.shape[0], dtype=torch.float64, device=device)
    for a in range(0, flat.shape[0], 1 << 18):
        g[a:a + (1 << 18)] = np.sqrt(2.0 / modes) * torch.cos(flat[a:a + (1 << 18)] @ om + ph).sum(dim=1)
    s = np.log(contrast) / float(g.max() - g.min())
    return torch.exp(s * g).reshape(shape)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    x = (x + np.uint64(0x9E3779B97F4A7C15)) & np.uint64(0xFFFFFFFFFFFFFFFF)
    z = x
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def hash_normal(points: np.ndarray, seed: int = 0) -> np.ndarray:
    """Pseudo-random N(0,1) values keyed by position (quantised to 2^-24).

    Two codes that number the same nodes differently get the same value at the same
    node, so random input vectors need no shared numbering.
    """
    with np.errstate(over="ignore"):
        q = np.round(np.asarray(points, dtype=np.float64) * (1 << 24)).astype(np.int64)
        q = q.view(np.uint64)
        h = _splitmix64(np.full(q.shape[:-1], np.uint64(seed), dtype=np.uint64))
        for d in range(q.shape[-1]):
            h = _splitmix64(h ^ q[..., d])
        h2 = _splitmix64(h)
    u1 = ((h >> np.uint64(11)).astype(np.float64) + 0.5) / float(1 << 53)
    u2 = ((h2 >> np.uint64(11)).astype(np.float64) + 0.5) / float(1 << 53)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def sine_solution(points: np.ndarray) -> np.ndarray:
    """u(x) = sin(pi x) sin(pi y) sin(pi z)."""
    return np.prod(np.sin(np.pi * points), axis=-1)


def sine_source(points: np.ndarray) -> np.ndarray:
    """f = -Laplace(u) = d pi^2 u for the sine solution in d = points.shape[-1] dimensions."""
    return np.asarray(points).shape[-1] * np.pi ** 2 * sine_solution(points)


def linear_patch(points: np.ndarray) -> np.ndarray:
    """u(x) = 1 + 2x - 3y + 0.5z, harmonic, used for the linear patch test."""
    return 1.0 + 2.0 * points[..., 0] - 3.0 * points[..., 1] + 0.5 * points[..., 2]


def uneven_mesh_list(count: int = 32, nmin: float = 1e4, nmax: float = 1e6,
                     orders=(2, 3, 4, 5, 6), seed: int = 4) -> list[dict]:
    """Sizes and orders of a batch of independent meshes of uneven size.

    Dof counts are log-uniform in [nmin, nmax], the order uniform over ``orders``;
    the lattice size is n = max(1, round((N^(1/3) - 1) / p)).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        ndof = float(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
        p = int(rng.choice(orders))
        n = max(1, int(round((ndof ** (1.0 / 3.0) - 1.0) / p)))
        out.append({"n": n, "p": p, "mesh_seed": 1000 + i})
    return out


def mlp_init(in_dim: int, hidden: int, out_dim: int, seed: int = 0,
             zero_last: bool = True) -> dict:
    """Initial weights of the element-patch network (He-normal hidden layers).

    The last layer starts at zero when ``zero_last`` (the preconditioner then
    starts as plain Jacobi).  W* are [out, in] row-major, float64.
    """
    rng = np.random.default_rng(seed)
    w1 = rng.normal(scale=np.sqrt(2.0 / in_dim), size=(hidden, in_dim))
    w2 = rng.normal(scale=np.sqrt(2.0 / hidden), size=(hidden, hidden))
    w3 = (np.zeros((out_dim, hidden)) if zero_last
          else rng.normal(scale=np.sqrt(1.0 / hidden), size=(out_dim, hidden)))
    return {"W1": w1, "b1": np.zeros(hidden), "W2": w2, "b2": np.zeros(hidden),
            "W3": w3, "b3": np.zeros(out_dim)}
