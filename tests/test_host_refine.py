"""Uniform refinement in the library (pafem_mesh_refine, host C++) against the oracle's
own refinement (oracle/pmg.py), on the CPU: the same vertices (matched by position),
the same connectivity in the same child order (8 e + o), and H1 spaces on the refined
meshes that agree with the oracle's dof for dof, element for element -- which on a
quadratic geometry also pins each child's 27 geometry nodes (dof positions come from
the element map)."""
import gc

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import synth
from oracle import pmg
from tests._common import match_by_coords

pafem = pytest.importorskip("paper_1911_09220_amd.pafem")

MESHES = {
    "jittered": lambda: synth.hex_lattice((2, 3, 2), 0.2, seed=3),
    "rotated": lambda: synth.hex_lattice(2, 0.15, seed=4, rotate_seed=5),
    "quadratic": lambda: synth.q2_warped_lattice(2, 0.05),
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_refinement_matches_oracle(name):
    mesh = MESHES[name]()
    ref = pmg.refine(mesh)
    F = pafem.Mesh.from_dict(mesh).refine()
    v, e = F.arrays()
    assert v.shape == ref["vertices"].shape and e.shape == ref["hex"].shape
    dist, idx = cKDTree(ref["vertices"]).query(v)
    assert dist.max() < 1e-13 and len(np.unique(idx)) == len(idx)
    np.testing.assert_array_equal(idx[e], ref["hex"])
    # coarse vertices keep their ids
    nv = mesh["vertices"].shape[0]
    np.testing.assert_array_equal(v[:nv], mesh["vertices"])


@pytest.mark.parametrize("name,p", [("jittered", 1), ("rotated", 2), ("quadratic", 3),
                                    ("rotated", 5)])
def test_spaces_on_refined_meshes_match_oracle(name, p):
    mesh = MESHES[name]()
    ref = pmg.refine(mesh)
    sp = pafem.Space(pafem.Mesh.from_dict(mesh).refine(), p, device=None)
    O = oracle.H1Space(ref, p)
    assert sp.ndofs == O.ndofs and sp.nelem == ref["hex"].shape[0]
    perm = match_by_coords(sp.dof_coords(), O.dof_coordinates())
    np.testing.assert_array_equal(perm[sp.elem_dofs()], O.elem_dofs)
    bd = np.zeros(sp.ndofs, dtype=bool)
    bd[sp.boundary_dofs()] = True
    np.testing.assert_array_equal(bd, O.boundary[perm])


def test_refining_twice_and_dropping_the_parent():
    mesh = synth.hex_lattice(1, 0.0)
    M = pafem.Mesh.from_dict(mesh)
    F = M.refine().refine()
    del M
    gc.collect()
    assert F.counts() == (125, 64)
    sp = pafem.Space(F, 2, device=None)
    assert sp.ndofs == 9 ** 3


def test_quadrilateral_refinement_is_refused():
    m = synth.quad_lattice(2, 0.0)
    with pytest.raises(pafem.PafemError):
        pafem.Mesh.from_dict(m).refine()


def test_refinement_entry_points_refuse_null_arguments():
    import ctypes as C
    lib = pafem.lib
    out = C.c_void_p()
    assert lib.pafem_mesh_refine(None, C.byref(out)) == -1          # EINVAL
    M = pafem.Mesh.from_dict(synth.hex_lattice(1))
    assert lib.pafem_mesh_refine(M.handle, None) == -1
    assert lib.pafem_mesh_info(None, None, None) == -1
    assert lib.pafem_mesh_vertices(None, None, None) == -1
    # either output may be omitted
    nv = C.c_int64()
    assert lib.pafem_mesh_info(M.handle, C.byref(nv), None) == 0 and nv.value == 8
    assert lib.pafem_mesh_vertices(M.handle, None, None) == 0
    # the coefficient mean across a refinement needs uploaded spaces on related meshes
    F = M.refine()
    Sc = pafem.Space(M, 1, device=None)
    Sf = pafem.Space(F, 1, device=None)
    assert lib.pafem_coeff_parent_mean(Sf.handle, Sc.handle, 0, None, 3, 3, None, None) != 0
