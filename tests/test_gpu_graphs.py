"""Graph replay of solver iterations against direct launches, and a caller's own
graph capture of the operator apply.

PCG batches and pairs of V-cycle FCG iterations are captured into HIP graphs once per
solve and replayed many times, with the host's own synchronisations and copies between
the replays.  Every solve is repeated with direct launches (pafem_set_graph_mode(0));
both must give the same iteration count (+-1, the atomic sums are unordered) and the
same solution to 1e-10, and repeated graph solves must agree with each other.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402


def _both(fn):
    """fn() under graph mode and under direct launches (graph mode restored)."""
    prev = P.pafem_set_graph_mode(1)
    try:
        g1 = fn()
        torch.cuda.synchronize()
        P.pafem_set_graph_mode(0)
        eager = fn()
        torch.cuda.synchronize()
        P.pafem_set_graph_mode(1)
        g2 = fn()
    finally:
        P.pafem_set_graph_mode(prev)
    return g1, eager, g2


def _close(a, b, tol=1e-10):
    return float((a - b).norm() / b.norm()) <= tol


@pytest.mark.parametrize("case", ["hex_p3", "hex_evec_p2", "quad_p1", "hex_mass_p2"])
def test_pcg_graph_replay_matches_direct_launches(case):
    if case.startswith("hex"):
        mesh = synth.hex_lattice(6, 0.1, seed=3, rotate_seed=4)
    else:
        mesh = synth.quad_lattice(40, 0.1, seed=3)
    p = int(case[-1])
    S = P.Space(P.Mesh.from_dict(mesh), p)
    kind = P.MASS if "mass" in case else P.DIFFUSION
    op = P.Operator(S, kind, S.qdata(kind), scatter="evec" if "evec" in case else "atomic")
    b = S.linear_form(P.SOURCE_SINE)
    for precond in (P.PRECOND_JACOBI, P.PRECOND_NONE):
        def solve():
            x, info = op.pcg(b, rel_tol=1e-11, max_iter=3000, precond=precond, check_every=8)
            return x, info
        (x1, i1), (xe, ie), (x2, i2) = _both(solve)
        print(f"{case} precond={precond}: graph {i1['iters']}/{i2['iters']} its, direct {ie['iters']}")
        assert i1["status"] == ie["status"] == i2["status"] == "OK"
        assert abs(i1["iters"] - ie["iters"]) <= 1 and abs(i2["iters"] - ie["iters"]) <= 1
        assert _close(x1, xe) and _close(x2, xe)
        k = min(len(i1["history"]), len(ie["history"]), 40)
        assert np.allclose(i1["history"][:k], ie["history"][:k], rtol=1e-8)


def test_pmg_fcg_graph_replay_matches_direct_launches():
    mesh = synth.hex_lattice(6, 0.1, seed=5)
    M = P.Mesh.from_dict(mesh)
    ops, diags, lmax = [], [], []
    for q in (4, 2, 1):
        S = P.Space(M, q)
        op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION))
        d = op.diagonal()
        v = torch.as_tensor(synth.hash_normal(S.dof_coords(), seed=q), device="cuda")
        ops.append(op)
        diags.append(d)
        lmax.append(op.lambda_max(d, v, 20))
    G = P.PMG(ops, diags, lmax, degree=2, coarse_iters=6)
    b = ops[0].space.linear_form(P.SOURCE_SINE)
    for check in (4, 5):
        def solve():
            return G.fcg(b, rel_tol=1e-10, max_iter=200, check_every=check)
        (x1, i1), (xe, ie), (x2, i2) = _both(solve)
        print(f"pmg check {check}: graph {i1['iters']}/{i2['iters']} its, direct {ie['iters']}")
        assert i1["status"] == ie["status"] == i2["status"] == "OK"
        assert abs(i1["iters"] - ie["iters"]) <= 1 and abs(i2["iters"] - ie["iters"]) <= 1
        assert _close(x1, xe) and _close(x2, xe)


@pytest.mark.parametrize("kind", ["diffusion", "mass_evec", "elasticity", "gradient"])
def test_caller_captures_apply_in_a_graph(kind):
    """A caller captures pafem_op_apply (its y-init is a kernel, not a memset) in a torch
    CUDA graph; every replay, with eager work and synchronisations between the replays
    (a new input written in place), equals the eager apply of the same input."""
    mesh = synth.hex_lattice(5, 0.1, seed=11, rotate_seed=12)
    S = P.Space(P.Mesh.from_dict(mesh), 3)
    X = S.dof_coords()
    if kind == "elasticity":
        E = S.nelem
        lm = torch.as_tensor(np.stack([np.full((E, 125), 1.5), np.full((E, 125), 0.7)], -1).ravel(),
                             device="cuda")
        op = P.Operator(S, P.ELASTICITY, S.qdata(P.ELASTICITY, coeff=lm))
        ncomp_in = ncomp_out = 3
    elif kind == "gradient":
        op = P.Operator(S, P.GRADIENT, S.qdata(P.GRADIENT), constrained=False)
        ncomp_in, ncomp_out = 1, 3
    else:
        k = P.DIFFUSION if kind == "diffusion" else P.MASS
        op = P.Operator(S, k, S.qdata(k), scatter="evec" if "evec" in kind else "atomic")
        ncomp_in = ncomp_out = 1

    def field(seed):
        v = np.concatenate([synth.hash_normal(X, seed=seed + c) for c in range(ncomp_in)])
        return torch.as_tensor(v, device="cuda")

    x = field(1)
    y = torch.empty(ncomp_out * S.ndofs, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        op.apply(x, y)                      # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        op.apply(x, y)
    for k in range(4):
        x.copy_(field(10 * (k + 2)))        # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        want = op.apply(x)
        torch.cuda.synchronize()
        assert _close(y, want, tol=1e-14), f"replay {k}"
