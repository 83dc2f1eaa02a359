"""GPU parity of the order-multigrid pieces against the CPU oracle (oracle/pmg.py).

Inputs are position-keyed (synth.hash_normal) on both sides and results are matched
by node position.  Bar: 1e-12 relative (FP64; only the summation order differs, the
atomic sums of restriction and apply included) for transfers, power iteration,
Chebyshev steps, element means and whole V-cycles (their coarse Jacobi-PCG
iterations included); the flexible CG with the V-cycle reaches the direct solution
and the oracle's iteration count +-2.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import forms, mlp, pmg
from tests._common import match_by_coords, rel_err, parity_err

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


@pytest.mark.parametrize("pc,pf", [(1, 1), (1, 2), (1, 3), (2, 3), (2, 4), (3, 6), (4, 8), (1, 8)])
def test_prolongation_and_restriction_match_oracle(pc, pf):
    mesh = _mesh(seed=pc + 10 * pf)
    M = P.Mesh.from_dict(mesh)
    Sc, Sf = P.Space(M, pc), P.Space(M, pf, renumber=True)
    Xc, Xf = Sc.dof_coords(), Sf.dof_coords()
    Po = pmg.interpolation(mesh, pc, pf)
    Oc, Of = oracle.H1Space(mesh, pc), oracle.H1Space(mesh, pf)
    pc_perm = match_by_coords(Xc, Oc.dof_coordinates())
    pf_perm = match_by_coords(Xf, Of.dof_coordinates())
    xc_o = synth.hash_normal(Oc.dof_coordinates(), seed=1)
    y = P.prolongate(Sc, Sf, _cuda(synth.hash_normal(Xc, seed=1))).cpu().numpy()
    want = (Po @ xc_o)[pf_perm]
    err = parity_err(y, want)
    print(f"prolongate {pc}->{pf}: rel err {err:.2e}")
    assert err <= TOL
    # add mode leaves essential entries alone
    y0 = _cuda(synth.hash_normal(Xf, seed=2))
    ya = P.prolongate(Sc, Sf, _cuda(synth.hash_normal(Xc, seed=1)), y0.clone(), add=True)
    assert parity_err(ya.cpu().numpy(), y0.cpu().numpy() + want) <= TOL
    # restriction: P^T (b - y)
    bo = synth.hash_normal(Of.dof_coordinates(), seed=3)
    yo = synth.hash_normal(Of.dof_coordinates(), seed=4)
    r = P.restrict(Sf, Sc, _cuda(synth.hash_normal(Xf, seed=3)),
                   _cuda(synth.hash_normal(Xf, seed=4))).cpu().numpy()
    want_r = (Po.T @ (bo - yo))[pc_perm]
    err = parity_err(r, want_r)
    print(f"restrict {pf}->{pc}: rel err {err:.2e}")
    assert err <= TOL
    r1 = P.restrict(Sf, Sc, _cuda(synth.hash_normal(Xf, seed=3))).cpu().numpy()
    assert parity_err(r1, (Po.T @ bo)[pc_perm]) <= TOL


def _levels_gpu(mesh, orders, kappa=None, mean=P.MEAN_ARITHMETIC, power_iters=20):
    M = P.Mesh.from_dict(mesh)
    E = mesh["hex"].shape[0]
    kc = None if kappa is None else _cuda(kappa.reshape(E, -1))
    spaces, ops, diags, lmax = [], [], [], []
    for l, p in enumerate(orders):
        S = P.Space(M, p)
        if kc is None:
            c = None
        elif l == 0:
            c = kc.reshape(-1).contiguous()
        else:
            c = S.coeff_mean(kc.reshape(-1).contiguous(), q1d_in=orders[0] + 2, q1d_out=p + 2,
                             kind=mean)
        op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION, coeff=c))
        d = op.diagonal()
        v = _cuda(synth.hash_normal(S.dof_coords(), seed=20 + p))
        spaces.append(S)
        ops.append(op)
        diags.append(d)
        lmax.append(op.lambda_max(d, v, power_iters))
    return M, spaces, ops, diags, lmax


def _levels_oracle(mesh, orders, kappa=None, mean="arithmetic", power_iters=20):
    starts = [synth.hash_normal(oracle.H1Space(mesh, p).dof_coordinates(), seed=20 + p)
              for p in orders]
    return pmg.build_levels(mesh, orders, kappa, mean, starts, power_iters)


def test_element_means_match_oracle():
    mesh = _mesh()
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, 5, 1.0, seed=3)
    S = P.Space(P.Mesh.from_dict(mesh), 3)
    for kind, name in ((P.MEAN_ARITHMETIC, "arithmetic"), (P.MEAN_GEOMETRIC, "geometric"),
                       (P.MEAN_HARMONIC, "harmonic")):
        got = S.coeff_mean(_cuda(kappa.reshape(-1)), q1d_in=5, q1d_out=3, kind=kind)
        got = got.cpu().numpy().reshape(E, 27)
        want = pmg.element_mean(kappa, name)
        np.testing.assert_allclose(got, np.repeat(want[:, None], 27, axis=1), rtol=1e-14)


@pytest.mark.parametrize("p", [1, 3, 5])
def test_power_iteration_and_chebyshev_match_oracle(p):
    mesh = _mesh(seed=p)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=4)
    _, spaces, ops, diags, lmax = _levels_gpu(mesh, [p], kappa, power_iters=12)
    levels, ospaces = _levels_oracle(mesh, [p], kappa, power_iters=12)
    print(f"p={p}: lmax gpu {lmax[0]:.15f} oracle {levels[0]['lmax']:.15f}")
    assert abs(lmax[0] - levels[0]["lmax"]) <= 1e-12 * levels[0]["lmax"]
    X = spaces[0].dof_coords()
    Xo = ospaces[0].dof_coordinates()
    perm = match_by_coords(X, Xo)
    A, d = levels[0]["A"], levels[0]["diag"]
    bo = synth.hash_normal(Xo, seed=7)
    b = _cuda(synth.hash_normal(X, seed=7))
    for degree in (1, 2, 3, 5):
        x = ops[0].chebyshev(diags[0], lmax[0], b, None, degree).cpu().numpy()
        want = pmg.chebyshev(A, d, bo, None, levels[0]["lmax"], degree)
        assert parity_err(x, want[perm]) <= TOL, degree
        x0o = synth.hash_normal(Xo, seed=8)
        x0 = _cuda(synth.hash_normal(X, seed=8))
        x = ops[0].chebyshev(diags[0], lmax[0], b, x0, degree, lo=0.2, hi=1.3).cpu().numpy()
        want = pmg.chebyshev(A, d, bo, x0o, levels[0]["lmax"], degree, lo=0.2, hi=1.3)
        assert parity_err(x, want[perm]) <= TOL, degree


@pytest.mark.parametrize("orders,coarse_iters", [([4, 2, 1], 0), ([4, 2, 1], 8), ([3, 1], 12),
                                                 ([2], 6), ([8, 4, 2, 1], 10)])
def test_vcycle_matches_oracle(orders, coarse_iters):
    mesh = _mesh((3, 3, 2), seed=5)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, orders[0] + 2, 1.0, seed=6)
    _, spaces, ops, diags, lmax = _levels_gpu(mesh, orders, kappa)
    levels, ospaces = _levels_oracle(mesh, orders, kappa)
    for l in range(len(orders)):
        assert abs(lmax[l] - levels[l]["lmax"]) <= 1e-12 * levels[l]["lmax"]
    G = P.PMG(ops, diags, lmax, degree=2, coarse_iters=coarse_iters)
    X = spaces[0].dof_coords()
    Xo = ospaces[0].dof_coordinates()
    perm = match_by_coords(X, Xo)
    z = G.vcycle(_cuda(synth.hash_normal(X, seed=9))).cpu().numpy()
    want = pmg.vcycle(levels, synth.hash_normal(Xo, seed=9), degree=2, coarse_iters=coarse_iters)
    err = parity_err(z, want[perm])
    print(f"vcycle {orders} coarse {coarse_iters}: rel err {err:.2e}")
    assert err <= TOL


def test_pmg_fcg_solves_and_matches_oracle_iterations():
    mesh = synth.hex_lattice(4, 0.1, seed=2)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, 6, 1.0, seed=5)
    orders = [4, 2, 1]
    _, spaces, ops, diags, lmax = _levels_gpu(mesh, orders, kappa)
    levels, ospaces = _levels_oracle(mesh, orders, kappa)
    G = P.PMG(ops, diags, lmax, degree=2, coarse_iters=10)
    b = spaces[0].linear_form(P.SOURCE_SINE)
    x, info = G.fcg(b, rel_tol=1e-10, max_iter=200)
    assert info["status"] == "OK" and info["converged"], info
    So = ospaces[0]
    bo = forms.assemble_vector(So, forms.element_load(mesh, 4, 6, synth.sine_source))
    bo[So.boundary] = 0.0
    A = levels[0]["A"]
    xo, k, _ = mlp.fcg(A, bo, lambda r: pmg.vcycle(levels, r, coarse_iters=10), tol=1e-10)
    perm = match_by_coords(spaces[0].dof_coords(), So.dof_coordinates())
    xd = spla.spsolve(A.tocsc(), bo)
    err = rel_err(x.cpu().numpy(), xd[perm])
    jac = oracle.pcg(A, bo, A.diagonal(), tol=1e-10)
    print(f"pmg fcg: gpu {info['iters']} its, oracle {k} its, jacobi {jac['iters']}; "
          f"rel err vs direct {err:.2e}")
    assert err <= 1e-8
    assert abs(info["iters"] - k) <= 2
    assert info["iters"] * 3 < jac["iters"]


def test_pmg_limits():
    mesh = _mesh()
    M1, M2 = P.Mesh.from_dict(mesh), P.Mesh.from_dict(mesh)
    S1, S2 = P.Space(M1, 1), P.Space(M2, 2)
    x = torch.zeros(S1.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PafemError):
        P.prolongate(S1, S2, x)        # different mesh objects
    S3 = P.Space(M1, 3)
    x3 = torch.zeros(S3.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PafemError):
        P.prolongate(S3, P.Space(M1, 2), x3)   # coarse order above fine order
    op = P.Operator(S3, P.DIFFUSION, S3.qdata(P.DIFFUSION), constrained=False)
    d = P.Operator(S3, P.DIFFUSION, S3.qdata(P.DIFFUSION)).diagonal()
    with pytest.raises(P.PafemError):
        P.PMG([op], [d], [1.0])         # levels must be constrained
    opc = P.Operator(S3, P.DIFFUSION, S3.qdata(P.DIFFUSION))
    with pytest.raises(P.PafemError):
        P.PMG([opc], [d], [-1.0])       # lmax must be positive
