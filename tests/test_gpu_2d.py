"""GPU parity of the quadrilateral (2D) path against the 2D oracle (oracle/twod.py).

Inputs are position-keyed (synth.hash_normal of the 2D node positions) on both sides
and results are matched by node position.  Bar: FP64 relative error <= 1e-12 for
applies, diagonals and load vectors; CG iteration histories equal to the oracle's
textbook CG up to roundoff.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import twod
from tests._common import match_by_coords, rel_err, parity_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402

TOL = 1e-12
# per order: several apply tiles (85, 64, 51, 42, 36, 32, 28, 25 elements) and a ragged last one
SHAPES = {1: (12, 9), 2: (10, 8), 3: (9, 7), 4: (8, 6), 5: (7, 6), 6: (7, 5), 7: (6, 5), 8: (7, 4)}


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _oracle(mesh, p, coeff=None, rho=None):
    S = twod.H1Space2D(mesh, p)
    K = oracle.assemble(S, twod.element_stiffness_2d(mesh, p, p + 2, coeff))
    M = oracle.assemble(S, twod.element_mass_2d(mesh, p, p + 2, rho))
    zero = np.zeros(S.ndofs)
    return S, oracle.constrain(K, zero, S.boundary)[0], oracle.constrain(M, zero, S.boundary)[0]


@pytest.mark.parametrize("p", range(1, 9))
def test_apply_2d(p):
    mesh = synth.quad_lattice(SHAPES[p], 0.1, seed=p, rotate_seed=40 + p)
    E = mesh["quad"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=7, dim=2)
    S = P.Space(P.Mesh.from_dict(mesh), p, renumber=(p % 2 == 1))
    X = S.dof_coords()
    So, Kc, Mc = _oracle(mesh, p, coeff=kappa, rho=kappa)
    perm = match_by_coords(X, So.dof_coordinates())
    xo = synth.hash_normal(So.dof_coordinates(), seed=p)
    x = _cuda(synth.hash_normal(X, seed=p))
    kc = _cuda(kappa.reshape(-1))
    for kind, A, name in ((P.DIFFUSION, Kc, "diffusion"), (P.MASS, Mc, "mass")):
        op = P.Operator(S, kind, S.qdata(kind, coeff=kc))
        y = op.apply(x).cpu().numpy()
        err = parity_err(y, (A @ xo)[perm])
        print(f"2D {name} p={p}: rel err {err:.2e}")
        assert err <= TOL
        d = op.diagonal().cpu().numpy()
        assert parity_err(d, A.diagonal()[perm]) <= TOL


@pytest.mark.parametrize("p,shape", [(1, (3, 2)), (2, (2, 2)), (3, (2, 1)), (6, (1, 1))])
def test_brute_force_columns_2d(p, shape):
    mesh = synth.quad_lattice(shape, 0.15, seed=3, rotate_seed=4)
    S = P.Space(P.Mesh.from_dict(mesh), p)
    So, Kc, _ = _oracle(mesh, p)
    op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION))
    n = S.ndofs
    A = np.empty((n, n))
    e = torch.zeros(n, dtype=torch.float64, device="cuda")
    for j in range(n):
        e.zero_()
        e[j] = 1.0
        A[:, j] = op.apply(e).cpu().numpy()
    perm = match_by_coords(S.dof_coords(), So.dof_coordinates())
    Aref = Kc.toarray()[np.ix_(perm, perm)]
    assert np.abs(A - Aref).max() <= TOL * np.abs(Aref).max()


@pytest.mark.parametrize("p", [1, 2, 4, 8])
def test_linear_form_and_cg_2d(p):
    """Load vector of the sine source; unpreconditioned CG (the paper's ex1 setting)
    follows the oracle's textbook CG residual history and reaches the direct solve."""
    mesh = synth.quad_lattice(SHAPES[p], 0.1, seed=10 + p)
    S = P.Space(P.Mesh.from_dict(mesh), p)
    So, Kc, _ = _oracle(mesh, p)
    perm = match_by_coords(S.dof_coords(), So.dof_coordinates())
    b = S.linear_form(P.SOURCE_SINE)
    bo = oracle.forms.assemble_vector(So, twod.element_load_2d(mesh, p, p + 2, synth.sine_source))
    bo[So.boundary] = 0.0
    assert parity_err(b.cpu().numpy(), bo[perm]) <= TOL
    op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION))
    x, info = op.pcg(b, rel_tol=1e-12, max_iter=3000, precond=P.PRECOND_NONE)
    assert info["status"] == "OK"
    r = oracle.pcg(Kc, bo, None, tol=1e-12, maxiter=3000)
    print(f"2D CG p={p}: {info['iters']} its (oracle {r['iters']})")
    assert abs(info["iters"] - r["iters"]) <= 2
    k = min(30, len(r["history"]), len(info["history"]))
    assert np.allclose(info["history"][:k], r["history"][:k], rtol=1e-8)
    xd = spla.spsolve(Kc.tocsc(), bo)
    assert rel_err(x.cpu().numpy(), xd[perm]) <= 1e-9
    xj, ij = op.pcg(b, rel_tol=1e-12, max_iter=3000)   # Jacobi
    assert ij["status"] == "OK" and rel_err(xj.cpu().numpy(), xd[perm]) <= 1e-9


def test_2d_limits():
    mesh = synth.quad_lattice(3, 0.1, seed=1)
    S = P.Space(P.Mesh.from_dict(mesh), 2)
    qd = S.qdata(P.DIFFUSION)
    with pytest.raises(P.PafemError):
        P.Operator(S, P.DIFFUSION, qd, scatter="evec")
    with pytest.raises(P.PafemError):
        P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, P.F32), qdata_dtype=P.F32)
    with pytest.raises(P.PafemError):
        S.qdata(P.DIFFUSION_GEOM)
    op = P.Operator(S, P.DIFFUSION, qd)
    with pytest.raises(P.PafemError):
        P.Batch([op], 2)
    with pytest.raises(P.PafemError):
        P.PMG([op], [op.diagonal()], [1.0])
