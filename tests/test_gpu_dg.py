"""GPU parity of the upwind DG convection on discontinuous spaces against the CPU
oracle (oracle/dg.py: element volume matrices, interior faces matched through shared
corners, outflow boundary faces, assembled sparse), through the C ABI.

Both sides number the DG dofs e * (p+1)^3 + i (caller element order, lexicographic
Gauss-Lobatto nodes), so vectors compare index by index.  Meshes are jittered with
scrambled element vertex orders (every face orientation occurs); inputs are values
keyed by node position and element.  Bar: ||got - want|| <= 1e-12 ||want|| and
max|got - want| <= 1e-12 max|want| (FP64).
"""
import numpy as np
import pytest

import synth
from oracle import dg
from tests._common import parity_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402  (must load: no fallback)

TOL = 1e-12
SHAPES = {1: (4, 4, 4), 2: (5, 4, 2), 3: (3, 3, 3), 4: (3, 3, 2), 5: (2, 2, 3),
          6: (3, 2, 1), 7: (2, 2, 2), 8: (3, 1, 1)}


def _x(mesh, p, seed):
    X = dg.dg_node_coordinates(mesh, p)
    E = mesh["hex"].shape[0]
    # node positions repeat across elements: mix in the element index
    tag = np.repeat(np.arange(E, dtype=np.float64), (p + 1) ** 3)[:, None] * 1e-3
    return synth.hash_normal(X + tag, seed=seed)


@pytest.mark.parametrize("beta", [(1.0, 0.5, 0.25), (-0.7, 0.4, -0.2)])
@pytest.mark.parametrize("p", range(1, 9))
def test_dg_convection_apply(p, beta):
    print(f"dg apply p={p} beta={beta}", flush=True)
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=20 + p, rotate_seed=60 + p)
    S = P.Space(P.Mesh.from_dict(mesh), p, family="l2")
    assert S.ndofs == mesh["hex"].shape[0] * (p + 1) ** 3 and S.nbdr == 0
    b = torch.tensor(beta, dtype=torch.float64, device="cuda")
    op = P.Operator(S, P.DG_CONVECTION, S.qdata(P.DG_CONVECTION, coeff=b), constrained=False)
    x = _x(mesh, p, p)
    got = op.apply(torch.as_tensor(x, device="cuda")).cpu().numpy()
    want = dg.dg_convection_matrix(mesh, p, p + 2, np.array(beta)) @ x
    err = parity_err(got, want)
    assert err <= TOL, (p, beta, err)


def test_dg_constant_field_gives_the_inflow_flux():
    """A 1 vanishes away from the inflow boundary and sums to minus the inflow flux, on a
    bench-shaped p = 3 lattice of 20^3 elements (every element and face)."""
    p = 3
    mesh = synth.hex_lattice(20, 0.05, seed=2)
    S = P.Space(P.Mesh.from_dict(mesh), p, family="l2")
    beta = np.array([1.0, 0.5, 0.25])
    op = P.Operator(S, P.DG_CONVECTION,
                    S.qdata(P.DG_CONVECTION, coeff=torch.tensor(beta, device="cuda")),
                    constrained=False)
    r = op.apply(torch.ones(S.ndofs, dtype=torch.float64, device="cuda")).cpu().numpy()
    X = S.dof_coords()
    inflow = np.any(np.abs(X) < 1e-12, axis=1)
    assert np.abs(r[~inflow]).max() < 1e-12
    assert abs(r.sum() - beta.sum()) < 1e-10


def test_dg_space_rejects_other_kinds():
    mesh = synth.hex_lattice(2, 0.0)
    S = P.Space(P.Mesh.from_dict(mesh), 2, family="l2")
    with pytest.raises(P.PafemError):
        S.qdata(P.DIFFUSION)
