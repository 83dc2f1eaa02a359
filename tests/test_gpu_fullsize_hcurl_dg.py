"""Parity of the H(curl) definite Maxwell apply and the upwind DG convection apply at
the sizes and in the launch configuration the benchmark times (~1e7 dofs per order,
5% jitter; Maxwell: lognormal (alpha, beta) per quadrature point, tangential
essential dofs eliminated; DG: constant velocity (1, 1/2, 1/4), zero inflow data).

The oracle cannot assemble 1e7-dof matrices, so it recomputes sampled outputs one by
one: for a few centre elements (two corners and random ones) it assembles its
operator on the 3x3x3 block of elements around the centre from scratch
(oracle/hcurl.py, oracle/dg.py).  Every element or face that touches a dof of the
centre element lies in that block, so the block's rows of those dofs are complete.
The sub-mesh keeps the global vertex numbers, so the Nedelec signs (set by global
vertex order on both sides) agree.  H(curl): dofs matched by node position, the
essential set from the positions (dofs on the cube's faces: y = x there, free rows
ignore essential columns), checked against the library's own list.  DG: dofs are
element-major on both sides (e * (p+1)^3 + i), inputs keyed by node position and
global element index.  Bar: essential outputs exact; free outputs within 1e-12
relative (2-norm and max-norm over the sampled outputs).
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth
from oracle import dg, hcurl
from tests._common import _patch, on_boundary, parity_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402  (must load: no fallback)

TARGET_DOFS = 1e7
TOL = 1e-12


def _centres(E, p, seed):
    rng = np.random.default_rng(seed)
    extra = 1 if p >= 6 else 2
    return [0, E - 1] + [int(c) for c in rng.integers(0, E, size=extra)]


@pytest.mark.parametrize("p", [1, 3, 6, 8])
def test_bench_size_hcurl_maxwell_on_sampled_rows(p):
    n = max(1, int(round((TARGET_DOFS / (3.0 * p ** 3)) ** (1.0 / 3.0))))
    mesh = synth.hex_lattice(n, 0.05, seed=2)
    E, q = mesh["hex"].shape[0], p + 2
    alpha = synth.lognormal_iid(E, q, 1.0, seed=4)
    beta = synth.lognormal_iid(E, q, 1.0, seed=5)
    S = P.Space(P.Mesh.from_dict(mesh), p, family="nd")
    N = S.ndofs
    print(f"hcurl p={p}: n={n}, {E} elements, {N} dofs", flush=True)
    assert 0.8e7 < N < 1.2e7
    Xlib = S.dof_coords()
    ess_lib = np.zeros(N, dtype=bool)
    ess_lib[S.boundary_dofs()] = True
    assert np.array_equal(ess_lib, on_boundary(Xlib))
    seed = 80 + p
    ab = torch.as_tensor(np.stack([alpha, beta], axis=-1), device="cuda").contiguous()
    op = P.Operator(S, P.HCURL_MAXWELL, S.qdata(P.HCURL_MAXWELL, coeff=ab))
    del ab
    y = op.apply(torch.as_tensor(synth.hash_normal(Xlib, seed=seed), device="cuda")).cpu().numpy()
    del op
    got, want, ess = [], [], []
    for c in _centres(E, p, 90 + p):
        ids, pos = _patch(n, c)
        sub = synth.sub_mesh(mesh, ids)
        ref = hcurl.NDSpace(sub, p)
        A = (hcurl.assemble_nd(ref, hcurl.element_nd_curlcurl(sub, p, q, alpha[ids])) +
             hcurl.assemble_nd(ref, hcurl.element_nd_mass(sub, p, q, beta[ids]))).tocsr()
        Xo = ref.dof_coordinates()
        eo = on_boundary(Xo)
        xo = synth.hash_normal(Xo, seed=seed)
        yo = np.where(eo, xo, A @ np.where(eo, 0.0, xo))
        dofs = ref.elem_dofs[pos]
        lo, hi = Xo[dofs].min(axis=0) - 1e-9, Xo[dofs].max(axis=0) + 1e-9
        cand = np.flatnonzero(np.all((Xlib >= lo) & (Xlib <= hi), axis=1))
        dist, idx = cKDTree(Xlib[cand]).query(Xo[dofs])
        assert dist.max() < 1e-10, "dof positions do not match"
        got.append(y[cand[idx]])
        want.append(yo[dofs])
        ess.append(eo[dofs])
    got, want, ess = np.concatenate(got), np.concatenate(want), np.concatenate(ess)
    err = parity_err(got[~ess], want[~ess])
    print(f"hcurl p={p}: sampled {len(got)} outputs ({int(ess.sum())} essential), "
          f"free rel err {err:.2e}", flush=True)
    assert np.array_equal(got[ess], want[ess])
    assert (~ess).sum() > 0 and err <= TOL


@pytest.mark.parametrize("p", [1, 3, 6, 8])
def test_bench_size_dg_convection_on_sampled_rows(p):
    n = max(1, int(round(TARGET_DOFS ** (1.0 / 3.0) / (p + 1))))
    mesh = synth.hex_lattice(n, 0.05, seed=2)
    E, nd = mesh["hex"].shape[0], (p + 1) ** 3
    S = P.Space(P.Mesh.from_dict(mesh), p, family="l2")
    N = S.ndofs
    print(f"dg p={p}: n={n}, {E} elements, {N} dofs", flush=True)
    assert N == E * nd and 0.8e7 < N < 1.2e7
    beta = np.array([1.0, 0.5, 0.25])
    seed = 100 + p
    Xlib = S.dof_coords()
    tag = np.repeat(np.arange(E, dtype=np.float64), nd)[:, None] * 1e-3
    x = synth.hash_normal(Xlib + tag, seed=seed)
    del tag
    op = P.Operator(S, P.DG_CONVECTION,
                    S.qdata(P.DG_CONVECTION, coeff=torch.tensor(beta, device="cuda")),
                    constrained=False)
    y = op.apply(torch.as_tensor(x, device="cuda")).cpu().numpy()
    del op
    got, want = [], []
    for c in _centres(E, p, 110 + p):
        ids, pos = _patch(n, c)
        sub = synth.sub_mesh(mesh, ids)
        A = dg.dg_convection_matrix(sub, p, p + 2, beta)
        Xo = dg.dg_node_coordinates(sub, p)
        assert np.abs(Xo[pos * nd:(pos + 1) * nd] - Xlib[c * nd:(c + 1) * nd]).max() < 1e-10
        to = np.repeat(np.asarray(ids, dtype=np.float64), nd)[:, None] * 1e-3
        yo = A @ synth.hash_normal(Xo + to, seed=seed)
        got.append(y[c * nd:(c + 1) * nd])
        want.append(yo[pos * nd:(pos + 1) * nd])
    got, want = np.concatenate(got), np.concatenate(want)
    err = parity_err(got, want)
    print(f"dg p={p}: sampled {len(got)} outputs, rel err {err:.2e}", flush=True)
    assert err <= TOL
