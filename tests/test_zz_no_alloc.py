"""pafem_op_apply_noalloc (the apply for callers that cannot allocate device memory)
against pafem_op_apply with a caller workspace, through the C ABI.

The deterministic scatter is bitwise reproducible, so with it both entry points must
give identical vectors; two calls in a row, the second on a smaller problem, check
that the library-held scratch is reused correctly.  The atomic scatter needs no
scratch and agrees to rounding.  An operator whose element vectors exceed the
scratch is refused before anything runs on the GPU.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402  (must load: no fallback)


def _problem(n, p, kind, seed):
    mesh = synth.hex_lattice(n, 0.1, seed=seed, rotate_seed=50 + seed)
    S = P.Space(P.Mesh.from_dict(mesh), p)
    x = torch.as_tensor(synth.hash_normal(S.dof_coords(), seed=seed), dtype=torch.float64,
                        device="cuda")
    return S, x


def test_noalloc_matches_workspace_apply_bitwise_twice():
    # first call: p = 3 on 6^3 elements (110 KB of element vectors per 16 elements);
    # second: smaller, p = 2 mass on 3 x 4 x 2 elements
    cases = [((6, 6, 6), 3, P.DIFFUSION, 1), ((3, 4, 2), 2, P.MASS, 2)]
    for n, p, kind, seed in cases:
        print(f"noalloc case n={n} p={p} kind={kind}", flush=True)
        S, x = _problem(n, p, kind, seed)
        op = P.Operator(S, kind, S.qdata(kind), scatter="evec")
        want = op.apply(x)
        got = torch.full_like(x, float("nan"))
        op.apply_noalloc(x, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (n, p, kind)
        assert np.isfinite(got.cpu().numpy()).all()


def test_noalloc_atomic_scatter_agrees_to_rounding():
    S, x = _problem((4, 3, 5), 4, P.DIFFUSION, 3)
    op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION))
    want = op.apply(x)
    got = torch.empty_like(x)
    op.apply_noalloc(x, got)
    torch.cuda.synchronize()
    err = (got - want).abs().max().item() / want.abs().max().item()
    assert err <= 1e-14, err


def test_noalloc_refuses_element_vectors_beyond_scratch():
    # p = 8: 729 element dofs * 8 B = 5832 B per element; 23^3 = 12167 elements need
    # 70.96 MB > 64 MiB.  The size check runs on the host before any launch.
    mesh = synth.hex_lattice((23, 23, 23))
    S = P.Space(P.Mesh.from_dict(mesh), 8)
    op = P.Operator(S, P.MASS, S.qdata(P.MASS), scatter="evec")
    x = torch.zeros(S.ndofs, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(P.PafemError) as ei:
        op.apply_noalloc(x, y)
    assert ei.value.code == -2 and "scratch" in str(ei.value)
    # the workspace entry point still serves the same operator
    op.apply(x, y)
    torch.cuda.synchronize()
    assert torch.count_nonzero(y).item() == 0
