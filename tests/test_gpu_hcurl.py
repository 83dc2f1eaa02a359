"""GPU parity of the H(curl) operators on Nedelec spaces against the CPU oracle
(oracle/hcurl.py: dense element matrices by quadrature, signed global assembly,
symmetric elimination of the tangential essential dofs), through the C ABI.

Both sides sign the global basis by the same rule on global vertex numbers (pinned on
the host in test_host_abi.py), so after matching dofs by node position the vectors
compare entry by entry.  Inputs are values keyed by node position
(``synth.hash_normal``) and seeded lognormal coefficients per quadrature point.  Bar:
||got - want|| <= 1e-12 ||want|| and max|got - want| <= 1e-12 max|want| (FP64).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import hcurl
from tests._common import match_by_coords, parity_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402  (must load: no fallback)

TOL = 1e-12

# per order: several element tiles (qdata_tile(p + 2) elements each) and a ragged last one
SHAPES = {1: (4, 4, 4), 2: (5, 4, 2), 3: (3, 3, 3), 4: (3, 3, 2), 5: (2, 2, 3),
          6: (3, 2, 1), 7: (2, 2, 2), 8: (3, 1, 1)}


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _setup(p, seed):
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=seed, rotate_seed=40 + seed)
    E, q = mesh["hex"].shape[0], p + 2
    alpha = synth.lognormal_iid(E, q, 1.0, seed=seed + 1)
    beta = synth.lognormal_iid(E, q, 1.0, seed=seed + 2)
    S = P.Space(P.Mesh.from_dict(mesh), p, family="nd")
    ref = hcurl.NDSpace(mesh, p)
    perm = match_by_coords(S.dof_coords(), ref.dof_coordinates())
    return mesh, alpha, beta, S, ref, perm


def _oracle_matrix(mesh, p, ref, kind, alpha, beta):
    q = p + 2
    if kind == P.HCURL_MASS:
        return hcurl.assemble_nd(ref, hcurl.element_nd_mass(mesh, p, q, beta))
    C = hcurl.assemble_nd(ref, hcurl.element_nd_curlcurl(mesh, p, q, alpha))
    if kind == P.HCURL_CURLCURL:
        return C
    return C + hcurl.assemble_nd(ref, hcurl.element_nd_mass(mesh, p, q, beta))


def _qdata(S, kind, alpha, beta):
    if kind == P.HCURL_MASS:
        return S.qdata(kind, coeff=_cuda(beta.ravel()))
    if kind == P.HCURL_CURLCURL:
        return S.qdata(kind, coeff=_cuda(alpha.ravel()))
    return S.qdata(kind, coeff=_cuda(np.stack([alpha, beta], axis=-1).ravel()))


@pytest.mark.parametrize("constrained", [True, False])
@pytest.mark.parametrize("kind", ["mass", "curlcurl", "maxwell"])
@pytest.mark.parametrize("p", range(1, 9))
def test_hcurl_apply(p, kind, constrained):
    k = {"mass": P.HCURL_MASS, "curlcurl": P.HCURL_CURLCURL, "maxwell": P.HCURL_MAXWELL}[kind]
    print(f"hcurl apply p={p} kind={kind} constrained={constrained}", flush=True)
    mesh, alpha, beta, S, ref, perm = _setup(p, 3 * p)
    A = _oracle_matrix(mesh, p, ref, k, alpha, beta)
    Xo = ref.dof_coordinates()
    xo = synth.hash_normal(Xo, seed=p)
    if constrained:
        A, _ = oracle.constrain(A, np.zeros(ref.ndofs), ref.boundary)
    want = A @ xo
    op = P.Operator(S, k, _qdata(S, k, alpha, beta), constrained=constrained)
    got = op.apply(_cuda(xo[perm])).cpu().numpy()
    err = parity_err(got, want[perm])
    assert err <= TOL, (p, kind, constrained, err)


def test_hcurl_curlcurl_annihilates_gradients():
    """The discrete gradient of an H1 function (the oracle's G, pinned on its own) lies in
    the null space of the GPU curl-curl operator, at p = 3 on a jittered mesh."""
    p = 3
    mesh = synth.hex_lattice((3, 3, 2), 0.1, seed=5, rotate_seed=6)
    S = P.Space(P.Mesh.from_dict(mesh), p, family="nd")
    ref = hcurl.NDSpace(mesh, p)
    G, spread = hcurl.discrete_gradient(ref, oracle.H1Space(mesh, p))
    assert spread < 1e-12
    perm = match_by_coords(S.dof_coords(), ref.dof_coordinates())
    phi = np.random.default_rng(1).normal(size=G.shape[1])
    u = G @ phi
    op = P.Operator(S, P.HCURL_CURLCURL, S.qdata(P.HCURL_CURLCURL), constrained=False)
    ku = op.apply(_cuda(u[perm])).cpu().numpy()
    opm = P.Operator(S, P.HCURL_MASS, S.qdata(P.HCURL_MASS), constrained=False)
    mu = opm.apply(_cuda(u[perm])).cpu().numpy()
    assert np.abs(ku).max() <= 1e-12 * np.abs(mu).max()


@pytest.mark.parametrize("p", [2, 4])
def test_hcurl_maxwell_cg_recovers_solution(p):
    """CG on the constrained definite Maxwell operator (the apply with its fused energy
    partials): b = A x_true from the GPU apply, solved back to x_true."""
    mesh, alpha, beta, S, ref, perm = _setup(p, 7 * p)
    op = P.Operator(S, P.HCURL_MAXWELL, _qdata(S, P.HCURL_MAXWELL, alpha, beta))
    X = S.dof_coords()
    xt = synth.hash_normal(X, seed=11)
    bd = S.boundary_dofs()
    xt[bd] = 0.0
    b = op.apply(_cuda(xt))
    x, info = op.pcg(b, rel_tol=1e-12, max_iter=4000, precond=P.PRECOND_NONE)
    assert info["status"] == "OK" and info["converged"], info
    err = np.linalg.norm(x.cpu().numpy() - xt) / np.linalg.norm(xt)
    assert err < 1e-8, err
