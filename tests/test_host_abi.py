"""CPU tests of the C-ABI library's host logic (no GPU calls).

* every symbol declared in include/pafem.h is exported by libpafem.so;
* the element->dof map, essential dofs and dof coordinates built by the C++
  host code agree exactly (integer for integer) with the oracle's independent
  numbering after matching dofs by position, including randomly rotated element
  vertex lists and the quadratic geometry;
* error statuses for bad input.
"""
import os
import re

import numpy as np
import pytest

import oracle
import synth
from tests._common import match_by_coords

pafem = pytest.importorskip("paper_1911_09220_amd.pafem",
                            reason="libpafem.so not built (run __graft_entry__.build())")

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "pafem.h")


def test_header_symbols_exported():
    text = open(HEADER).read()
    names = set(re.findall(r"\b(pafem_[a-z0-9_]+)\s*\(", text))
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(pafem.lib, n), f"{n} declared in pafem.h but not exported"


@pytest.mark.parametrize("case", [
    ("lattice", 1, False), ("lattice", 2, False), ("lattice", 3, True), ("lattice", 4, False),
    ("rotated", 2, False), ("rotated", 3, False), ("rotated", 5, True), ("q2", 2, False),
    ("q2", 3, True), ("rotated", 8, False)])
def test_element_dof_map_matches_oracle(case):
    kind, p, renumber = case
    if kind == "lattice":
        mesh = synth.hex_lattice(3, 0.1, seed=3)
    elif kind == "rotated":
        mesh = synth.hex_lattice(3, 0.1, seed=4, rotate_seed=17)
    else:
        mesh = synth.q2_warped_lattice(2)
    sp = pafem.Space(pafem.Mesh.from_dict(mesh), p, renumber=renumber, device=None)
    ref = oracle.H1Space(mesh, p)
    assert sp.ndofs == ref.ndofs and sp.nelem == mesh["hex"].shape[0]
    assert sp.dofs_per_elem == (p + 1) ** 3
    X = sp.dof_coords()
    perm = match_by_coords(X, ref.dof_coordinates())      # lib dof i <-> oracle dof perm[i]
    assert len(np.unique(perm)) == sp.ndofs
    gmap = sp.elem_dofs()
    np.testing.assert_array_equal(perm[gmap], ref.elem_dofs)
    bd = np.zeros(sp.ndofs, dtype=bool)
    bd[sp.boundary_dofs()] = True
    np.testing.assert_array_equal(bd, ref.boundary[perm])
    assert sp.nbdr == ref.boundary.sum()


def test_default_numbering_order():
    """Vertex dofs first, then edges, faces, interiors (the paper's global order)."""
    mesh = synth.hex_lattice(2, 0.0)
    sp = pafem.Space(pafem.Mesh.from_dict(mesh), 3, device=None)
    ref = oracle.H1Space(mesh, 3)
    perm = match_by_coords(sp.dof_coords(), ref.dof_coordinates())
    cls = ref.dof_class[perm]              # class of lib dof i
    assert np.all(np.diff(cls) >= 0)


def test_bad_inputs():
    mesh = synth.hex_lattice(2)
    bad = mesh["hex"].copy()
    bad[0, 0] = 10_000
    with pytest.raises(pafem.PafemError) as ei:
        pafem.Mesh(mesh["vertices"], bad)
    assert ei.value.code == -1
    rep = mesh["hex"].copy()
    rep[1, 3] = rep[1, 0]
    with pytest.raises(pafem.PafemError):
        pafem.Mesh(mesh["vertices"], rep)
    m = pafem.Mesh.from_dict(mesh)
    with pytest.raises(pafem.PafemError) as ei:
        pafem.Space(m, 9, device=None)
    assert ei.value.code == -3
    # three elements on one face: not conforming
    h = np.concatenate([mesh["hex"], mesh["hex"][:1]], axis=0)
    with pytest.raises(pafem.PafemError) as ei:
        pafem.Space(pafem.Mesh(mesh["vertices"], h), 1, device=None)
    assert ei.value.code == -1
    with pytest.raises(pafem.PafemError):
        pafem.Mesh(mesh["vertices"], mesh["hex"], geom_order=2)   # nodes missing


@pytest.mark.parametrize("p,rotate,renumber", [(1, False, False), (2, True, False), (3, True, True),
                                                (4, False, False), (8, True, False)])
def test_quad_element_dof_map_matches_oracle(p, rotate, renumber):
    from oracle import twod
    mesh = synth.quad_lattice((4, 3), 0.1, seed=5, rotate_seed=9 if rotate else None)
    sp = pafem.Space(pafem.Mesh.from_dict(mesh), p, renumber=renumber, device=None)
    ref = twod.H1Space2D(mesh, p)
    assert sp.dim == 2 and sp.ndofs == ref.ndofs and sp.dofs_per_elem == (p + 1) ** 2
    X = sp.dof_coords()
    assert X.shape == (sp.ndofs, 2)
    perm = match_by_coords(X, ref.dof_coordinates())
    assert len(np.unique(perm)) == sp.ndofs
    np.testing.assert_array_equal(perm[sp.elem_dofs()], ref.elem_dofs)
    bd = np.zeros(sp.ndofs, dtype=bool)
    bd[sp.boundary_dofs()] = True
    np.testing.assert_array_equal(bd, ref.boundary[perm])
    if not renumber:
        cls = ref.dof_class[perm]          # vertices, then edges, then interiors
        assert np.all(np.diff(cls) >= 0)


def test_empty_mesh_rejected():
    with pytest.raises(pafem.PafemError) as ei:
        pafem.Mesh(np.zeros((8, 3)), np.zeros((0, 8), dtype=np.int64))
    assert ei.value.code == -1


@pytest.mark.parametrize("p", [1, 3, 8])
def test_qdata_sizes_per_kind(p):
    """Values per point of every operator kind, padded to whole apply tiles of
    floor(256 / Q^2) elements; unknown kinds and q1d outside the tables are refused."""
    mesh = synth.hex_lattice((3, 2, 2), 0.1, seed=4)
    S = pafem.Space(pafem.Mesh.from_dict(mesh), p, device=None)
    Q = p + 2
    nt = max(1, 256 // (Q * Q))
    tiles = -(-S.nelem // nt)
    per_point = {pafem.MASS: 1, pafem.DIFFUSION: 6, pafem.DIFFUSION_GEOM: 1, pafem.CONVECTION: 3,
                 pafem.GRADIENT: 9, pafem.DIVERGENCE: 9, pafem.ELASTICITY: 11}
    for kind, nc in per_point.items():
        assert pafem.pafem_qdata_size(S.handle, kind, Q) == tiles * nt * nc * Q ** 3
    for bad_kind in (-1, 7, 16, 17):
        with pytest.raises(pafem.PafemError):
            pafem.pafem_qdata_size(S.handle, bad_kind, Q)
    with pytest.raises(pafem.PafemError):
        pafem.pafem_qdata_size(S.handle, pafem.DIFFUSION, 13)


@pytest.mark.parametrize("case", [
    ("lattice", 1, False), ("lattice", 2, False), ("rotated", 2, False), ("rotated", 3, True),
    ("rotated", 4, False), ("q2", 2, False), ("q2", 3, True), ("rotated", 6, False)])
def test_nedelec_numbering_and_signs_match_oracle(case):
    """The library's Nedelec space against the oracle's (oracle/hcurl.py): same dofs
    (matched by node position), same element maps, the same orientation sign of every
    element-local dof and the same essential set."""
    from oracle import hcurl
    kind, p, renumber = case
    if kind == "lattice":
        mesh = synth.hex_lattice((3, 2, 2), 0.1, seed=3)
    elif kind == "rotated":
        mesh = synth.hex_lattice((2, 3, 2), 0.1, seed=4, rotate_seed=17)
    else:
        mesh = synth.q2_warped_lattice(2)
    sp = pafem.Space(pafem.Mesh.from_dict(mesh), p, renumber=renumber, device=None, family="nd")
    ref = hcurl.NDSpace(mesh, p)
    assert sp.ndofs == ref.ndofs and sp.dofs_per_elem == 3 * p * (p + 1) ** 2
    perm = match_by_coords(sp.dof_coords(), ref.dof_coordinates())
    assert len(np.unique(perm)) == sp.ndofs
    np.testing.assert_array_equal(perm[sp.elem_dofs()], ref.elem_dofs)
    np.testing.assert_array_equal(sp.elem_signs(), ref.elem_signs.astype(np.int8))
    bd = np.zeros(sp.ndofs, dtype=bool)
    bd[sp.boundary_dofs()] = True
    np.testing.assert_array_equal(bd, ref.boundary[perm])
