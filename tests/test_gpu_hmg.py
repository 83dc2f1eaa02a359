"""GPU parity of multigrid in the mesh size (h-multigrid) against the CPU oracle
(oracle/pmg.py: refine, h_interpolation, level_coefficient, build_hp_levels).

Meshes are refined by the library (pafem_mesh_refine) and by the oracle
independently; inputs are position-keyed (synth.hash_normal) on both sides and results
are matched by node position.  Bar as for the order multigrid: 1e-12 relative (FP64;
only the summation order differs, the restriction's and the apply's atomic sums
included) for transfers, coefficient means and whole V-cycles; the flexible CG reaches
the direct solution and the oracle's iteration count +-2.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import forms, mlp, pmg
from tests._common import match_by_coords, parity_err, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402

TOL = 1e-12


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _mesh(shape=(3, 2, 2), seed=1):
    return synth.hex_lattice(shape, 0.1, seed=seed, rotate_seed=seed + 50)


@pytest.mark.parametrize("pc,pf", [(1, 1), (1, 2), (2, 2), (2, 3), (3, 3), (3, 6), (4, 8),
                                   (8, 8)])
def test_h_prolongation_and_restriction_match_oracle(pc, pf):
    mesh = _mesh(seed=pc + 10 * pf)
    fine = pmg.refine(mesh)
    Mc = P.Mesh.from_dict(mesh)
    Mf = Mc.refine()
    Sc, Sf = P.Space(Mc, pc), P.Space(Mf, pf, renumber=True)
    Xc, Xf = Sc.dof_coords(), Sf.dof_coords()
    Oc, Of = oracle.H1Space(mesh, pc), oracle.H1Space(fine, pf)
    Po = pmg.h_interpolation(mesh, fine, pc, pf)
    pc_perm = match_by_coords(Xc, Oc.dof_coordinates())
    pf_perm = match_by_coords(Xf, Of.dof_coordinates())
    xc_o = synth.hash_normal(Oc.dof_coordinates(), seed=1)
    y = P.prolongate(Sc, Sf, _cuda(synth.hash_normal(Xc, seed=1))).cpu().numpy()
    want = (Po @ xc_o)[pf_perm]
    err = parity_err(y, want)
    print(f"h-prolongate {pc}->{pf}: rel err {err:.2e}")
    assert err <= TOL
    y0 = _cuda(synth.hash_normal(Xf, seed=2))
    ya = P.prolongate(Sc, Sf, _cuda(synth.hash_normal(Xc, seed=1)), y0.clone(), add=True)
    assert parity_err(ya.cpu().numpy(), y0.cpu().numpy() + want) <= TOL
    bo = synth.hash_normal(Of.dof_coordinates(), seed=3)
    yo = synth.hash_normal(Of.dof_coordinates(), seed=4)
    r = P.restrict(Sf, Sc, _cuda(synth.hash_normal(Xf, seed=3)),
                   _cuda(synth.hash_normal(Xf, seed=4))).cpu().numpy()
    want_r = (Po.T @ (bo - yo))[pc_perm]
    err = parity_err(r, want_r)
    print(f"h-restrict {pf}->{pc}: rel err {err:.2e}")
    assert err <= TOL


def test_two_refinements_and_a_quadratic_geometry():
    """Transfers across two refinements in a row (the element order is inherited
    twice) and on a quadratic geometry (the children carry the parent's map)."""
    for mesh in (synth.hex_lattice((2, 1, 1), 0.15, seed=7, rotate_seed=8),
                 synth.q2_warped_lattice(2, 0.05)):
        m1 = pmg.refine(mesh)
        m2 = pmg.refine(m1)
        M0 = P.Mesh.from_dict(mesh)
        M1 = M0.refine()
        M2 = M1.refine()
        S1, S2 = P.Space(M1, 2), P.Space(M2, 3)
        O1, O2 = oracle.H1Space(m1, 2), oracle.H1Space(m2, 3)
        X1, X2 = S1.dof_coords(), S2.dof_coords()
        p1 = match_by_coords(X1, O1.dof_coordinates())
        p2 = match_by_coords(X2, O2.dof_coordinates())
        Po = pmg.h_interpolation(m1, m2, 2, 3)
        y = P.prolongate(S1, S2, _cuda(synth.hash_normal(X1, seed=5))).cpu().numpy()
        want = (Po @ synth.hash_normal(O1.dof_coordinates(), seed=5))[p2]
        assert parity_err(y, want) <= TOL
        r = P.restrict(S2, S1, _cuda(synth.hash_normal(X2, seed=6))).cpu().numpy()
        assert parity_err(r, (Po.T @ synth.hash_normal(O2.dof_coordinates(), seed=6))[p1]) <= TOL
        # transfers skip no generation
        S0 = P.Space(M0, 1)
        with pytest.raises(P.PafemError):
            P.prolongate(S0, S2, torch.zeros(S0.ndofs, dtype=torch.float64, device="cuda"))


def test_parent_means_match_oracle():
    mesh = _mesh()
    M = P.Mesh.from_dict(mesh)
    F = M.refine()
    Sc, Sf = P.Space(M, 1), P.Space(F, 3)
    Ef = 8 * mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(Ef, 5, 1.0, seed=3)
    for kind, name in ((P.MEAN_ARITHMETIC, "arithmetic"), (P.MEAN_GEOMETRIC, "geometric"),
                       (P.MEAN_HARMONIC, "harmonic")):
        got = Sf.coeff_parent_mean(Sc, _cuda(kappa.reshape(-1)), q1d_in=5, q1d_out=3, kind=kind)
        want = pmg.level_coefficient(kappa, Ef // 8, 3, name)
        np.testing.assert_allclose(got.cpu().numpy().reshape(-1, 27), want, rtol=1e-14)
    with pytest.raises(P.PafemError):
        Sc.coeff_parent_mean(Sf, _cuda(np.ones(Sc.nelem * 27)), q1d_in=3, q1d_out=5)


def _hp_gpu(mesh_dicts, plan, kappa=None, power_iters=20):
    """Library levels: meshes[k] = refinement of meshes[k+1], built by the library."""
    meshes = [P.Mesh.from_dict(mesh_dicts[-1])]
    for _ in range(len(mesh_dicts) - 1):
        meshes.insert(0, meshes[0].refine())
    spaces, ops, diags, lmax = [], [], [], []
    c_prev = None
    for l, (m, p) in enumerate(plan):
        S = P.Space(meshes[m], p)
        if kappa is None:
            c = None
        elif l == 0:
            c = _cuda(kappa.reshape(-1))
        elif plan[l - 1][0] == m:
            # same mesh: the previous level's coefficient is constant per element
            c = spaces[-1].coeff_mean(c_prev, q1d_in=plan[l - 1][1] + 2, q1d_out=p + 2)
        else:
            c = spaces[-1].coeff_parent_mean(S, c_prev, q1d_in=plan[l - 1][1] + 2, q1d_out=p + 2)
        op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION, coeff=c))
        d = op.diagonal()
        v = _cuda(synth.hash_normal(S.dof_coords(), seed=40 + l))
        spaces.append(S)
        ops.append(op)
        diags.append(d)
        lmax.append(op.lambda_max(d, v, power_iters))
        c_prev = c
    return meshes, spaces, ops, diags, lmax


def _hp_oracle(mesh_dicts, plan, kappa=None, power_iters=20):
    starts = [synth.hash_normal(oracle.H1Space(mesh_dicts[m], p).dof_coordinates(), seed=40 + l)
              for l, (m, p) in enumerate(plan)]
    return pmg.build_hp_levels(mesh_dicts, plan, kappa, "arithmetic", starts, power_iters)


def _chain(coarse, n):
    out = [coarse]
    for _ in range(n):
        out.insert(0, pmg.refine(out[0]))
    return out


@pytest.mark.parametrize("plan,coarse_iters", [
    ([(0, 1), (1, 1)], 0), ([(0, 1), (1, 1)], 6), ([(0, 3), (0, 1), (1, 1)], 8),
    ([(0, 2), (1, 2), (1, 1)], 10), ([(0, 4), (0, 2), (1, 1), (2, 1)], 5)])
def test_hp_vcycle_matches_oracle(plan, coarse_iters):
    nmesh = plan[-1][0] + 1
    # the coarsest mesh keeps free dofs at p = 1 (two interior vertices)
    dicts = _chain(synth.hex_lattice((3, 2, 2), 0.1, seed=5, rotate_seed=6), nmesh - 1)
    E = dicts[0]["hex"].shape[0]
    kappa = synth.lognormal_iid(E, plan[0][1] + 2, 1.0, seed=6)
    _, spaces, ops, diags, lmax = _hp_gpu(dicts, plan, kappa)
    levels, ospaces = _hp_oracle(dicts, plan, kappa)
    for l in range(len(plan)):
        assert abs(lmax[l] - levels[l]["lmax"]) <= 1e-12 * levels[l]["lmax"], l
    G = P.PMG(ops, diags, lmax, degree=2, coarse_iters=coarse_iters)
    X, Xo = spaces[0].dof_coords(), ospaces[0].dof_coordinates()
    perm = match_by_coords(X, Xo)
    z = G.vcycle(_cuda(synth.hash_normal(X, seed=9))).cpu().numpy()
    want = pmg.vcycle(levels, synth.hash_normal(Xo, seed=9), degree=2, coarse_iters=coarse_iters)
    err = parity_err(z, want[perm])
    print(f"hp vcycle {plan} coarse {coarse_iters}: rel err {err:.2e}")
    assert err <= TOL


def test_hp_fcg_solves_and_matches_oracle_iterations():
    dicts = _chain(synth.hex_lattice(2, 0.1, seed=6), 2)
    E = dicts[0]["hex"].shape[0]
    kappa = synth.lognormal_iid(E, 4, 1.0, seed=5)
    plan = [(0, 2), (0, 1), (1, 1), (2, 1)]
    _, spaces, ops, diags, lmax = _hp_gpu(dicts, plan, kappa)
    levels, ospaces = _hp_oracle(dicts, plan, kappa)
    G = P.PMG(ops, diags, lmax, degree=2, coarse_iters=10)
    b = spaces[0].linear_form(P.SOURCE_SINE)
    x, info = G.fcg(b, rel_tol=1e-10, max_iter=200)
    assert info["status"] == "OK" and info["converged"], info
    So = ospaces[0]
    bo = forms.assemble_vector(So, forms.element_load(dicts[0], 2, 4, synth.sine_source))
    bo[So.boundary] = 0.0
    A = levels[0]["A"]
    xo, k, _ = mlp.fcg(A, bo, lambda r: pmg.vcycle(levels, r, coarse_iters=10), tol=1e-10)
    perm = match_by_coords(spaces[0].dof_coords(), So.dof_coordinates())
    xd = spla.spsolve(A.tocsc(), bo)
    err = rel_err(x.cpu().numpy(), xd[perm])
    jac = oracle.pcg(A, bo, A.diagonal(), tol=1e-10)
    print(f"hp fcg: gpu {info['iters']} its, oracle {k} its, jacobi {jac['iters']}; "
          f"rel err vs direct {err:.2e}")
    assert err <= 1e-8
    assert abs(info["iters"] - k) <= 2
    assert info["iters"] * 3 < jac["iters"]


def test_transfers_refuse_unrelated_meshes():
    mesh = _mesh()
    M = P.Mesh.from_dict(mesh)
    F = M.refine()
    other = P.Mesh.from_dict(mesh)          # same arrays, another object
    Sf = P.Space(F, 1)
    So = P.Space(other, 1)
    x = torch.zeros(So.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PafemError):
        P.prolongate(So, Sf, x)
    Sc = P.Space(M, 1)
    xf = torch.zeros(Sf.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PafemError):
        P.prolongate(Sf, Sc, xf)            # the refined space is not the coarse one
    y = P.prolongate(Sc, Sf, torch.ones(Sc.ndofs, dtype=torch.float64, device="cuda"))
    free = torch.ones(Sf.ndofs, dtype=torch.float64, device="cuda")
    free[torch.as_tensor(Sf.boundary_dofs(), device="cuda").long()] = 0.0
    assert torch.equal(y * free, y)
    # on free dofs away from the boundary the constant prolongates to itself
    interior = P.restrict(Sf, Sc, free).cpu().numpy()
    assert np.all(interior >= 0.0)
