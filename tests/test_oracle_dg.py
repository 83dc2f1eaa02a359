"""Pins of the upwind DG convection oracle (oracle/dg.py).

* Affine lattices, piecewise-linear discontinuous fields u|_K = c_K + g_K . (x - x_K):
  w^T A u equals the integrals of the form evaluated directly in physical space --
  volume -int u beta . grad w, upwind traces on every interior face, outflow boundary
  faces -- with faces found from element positions, not from the reference element.
  Element vertex orders are scrambled, so the face matching of the oracle is exercised.
* Jittered meshes, constant velocity: A 1 vanishes away from the inflow boundary and
  sums to minus the inflow flux (beta_x + beta_y + beta_z on the unit cube).
* Continuous fields (the H1 space injected, the same Gauss-Lobatto nodes): rows of test
  functions vanishing on the inflow boundary equal the H1 convection matrix (the
  divergence theorem, exact for these quadrature degrees on trilinear elements).
* The symmetric part is positive semidefinite (upwinding dissipates).
A wrong upwind side, a flipped normal, a mismatched face orientation or a dropped face
term breaks one of these.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import dg, forms

BETA = np.array([1.0, 0.5, 0.25])


def _piecewise_linear(mesh, n, seed):
    """Per-element (c_K, g_K, x_K) and the DG dofs of u|_K = c_K + g_K . (x - x_K)."""
    rng = np.random.default_rng(seed)
    E = mesh["hex"].shape[0]
    c = rng.normal(size=E)
    g = rng.normal(size=(E, 3))
    xc = mesh["vertices"][mesh["hex"]].mean(axis=1)
    return c, g, xc


def _dofs(mesh, p, c, g, xc):
    X = dg.dg_node_coordinates(mesh, p).reshape(len(c), -1, 3)
    return (c[:, None] + np.einsum("ea,eka->ek", g, X - xc[:, None, :])).ravel()


def _physical_form(n, cu, gu, cw, gw, xc, beta):
    """a(u, w) on the axis-aligned lattice n^3 of the unit cube, straight from the
    definition with 2-point Gauss rules on each physical face."""
    h = 1.0 / n
    idx = np.floor(xc / h).astype(int)                       # lattice position of each element
    at = {tuple(v): e for e, v in enumerate(idx.tolist())}
    total = -np.sum((gw @ beta) * cu) * h ** 3               # volume: int (x - x_K) = 0
    g1 = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    for key, e in at.items():
        for a in range(3):
            b, c2 = [d for d in range(3) if d != a]
            pts = []
            for s in g1:
                for t in g1:
                    x = np.empty(3)
                    x[a] = (key[a] + 1) * h
                    x[b] = (key[b] + s) * h
                    x[c2] = (key[c2] + t) * h
                    pts.append(x)
            pts = np.array(pts)
            wq = h * h / 4.0
            val = lambda cc, gg, k: cc[k] + (pts - xc[k]) @ gg[k]
            nb = list(key)
            nb[a] += 1
            bn = beta[a]                                         # n = +e_a
            um, wm = val(cu, gu, e), val(cw, gw, e)
            if tuple(nb) in at:
                f = at[tuple(nb)]
                up, wp = val(cu, gu, f), val(cw, gw, f)
                uup = um if bn > 0 else up
                total += wq * np.sum(bn * uup * (wm - wp))
            elif bn > 0:                                         # outflow face x_a = 1
                total += wq * np.sum(bn * um * wm)
            # the face x_a = key[a] h of an element on the low boundary: inflow for bn > 0
            if key[a] == 0 and bn < 0:
                lo = pts.copy()
                lo[:, a] = 0.0
                total += wq * np.sum(-bn * (cu[e] + (lo - xc[e]) @ gu[e]) *
                                     (cw[e] + (lo - xc[e]) @ gw[e]))
    return total


@pytest.mark.parametrize("p", [1, 2, 3])
def test_form_on_piecewise_linear_fields_matches_physical_integrals(p):
    n = 3
    mesh = synth.hex_lattice(n, 0.0, seed=0, rotate_seed=11 + p)
    cu, gu, xc = _piecewise_linear(mesh, n, 1)
    cw, gw, _ = _piecewise_linear(mesh, n, 2)
    A = dg.dg_convection_matrix(mesh, p, p + 2, BETA)
    got = _dofs(mesh, p, cw, gw, xc) @ (A @ _dofs(mesh, p, cu, gu, xc))
    want = _physical_form(n, cu, gu, cw, gw, xc, BETA)
    assert abs(got - want) < 1e-12 * max(1.0, abs(want))


def test_form_with_a_negative_velocity_component():
    n, p = 3, 2
    beta = np.array([-0.7, 0.4, -0.2])
    mesh = synth.hex_lattice(n, 0.0, seed=0, rotate_seed=5)
    cu, gu, xc = _piecewise_linear(mesh, n, 3)
    cw, gw, _ = _piecewise_linear(mesh, n, 4)
    A = dg.dg_convection_matrix(mesh, p, p + 2, beta)
    got = _dofs(mesh, p, cw, gw, xc) @ (A @ _dofs(mesh, p, cu, gu, xc))
    want = _physical_form(n, cu, gu, cw, gw, xc, beta)
    assert abs(got - want) < 1e-12 * max(1.0, abs(want))


@pytest.mark.parametrize("p", [1, 3])
def test_constant_field_gives_the_inflow_flux(p):
    mesh = synth.hex_lattice((3, 2, 2), 0.15, seed=3, rotate_seed=4)
    A = dg.dg_convection_matrix(mesh, p, p + 2, BETA)
    r = A @ np.ones(A.shape[0])
    X = dg.dg_node_coordinates(mesh, p)
    inflow = np.any(np.abs(X) < 1e-12, axis=1)               # faces x = 0, y = 0, z = 0
    assert np.abs(r[~inflow]).max() < 1e-13
    assert abs(r.sum() - BETA.sum()) < 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_continuous_fields_reduce_to_h1_convection(p):
    mesh = synth.hex_lattice((2, 3, 2), 0.12, seed=6, rotate_seed=7)
    H = oracle.H1Space(mesh, p)
    Ch = oracle.assemble(H, forms.element_convection(mesh, p, p + 2, BETA)).toarray()
    A = dg.dg_convection_matrix(mesh, p, p + 2, BETA).toarray()
    Pm = np.zeros((A.shape[0], H.ndofs))
    Pm[np.arange(A.shape[0]), H.elem_dofs.ravel()] = 1.0      # DG dof (e, i) = H1 dof of node i
    red = Pm.T @ A @ Pm
    Xh = H.dof_coordinates()
    keep = ~np.any(np.abs(Xh) < 1e-12, axis=1)               # test functions zero on inflow faces
    assert np.abs(red[keep] - Ch[keep]).max() < 1e-13 * np.abs(Ch).max()
    assert np.abs(red[~keep] - Ch[~keep]).max() > 1e-6      # the inflow rows do differ


@pytest.mark.parametrize("p", [1, 2])
def test_symmetric_part_is_positive_semidefinite(p):
    mesh = synth.hex_lattice((2, 2, 2), 0.15, seed=8, rotate_seed=9)
    A = dg.dg_convection_matrix(mesh, p, p + 2, BETA).toarray()
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() > -1e-12 * np.abs(ev).max()
    assert ev.max() > 0.0
