"""Batched multi-right-hand-side apply over uneven meshes (one graph launch).

Each column of the batched result is compared with the single-vector FP64 apply
of its mesh (which is itself parity-checked against the oracle), every tile
candidate gives the same result, graph replays interleaved with other work all
match the eager result, and one small mesh is checked against the oracle
directly.  Bars: FP64 1e-12 relative, FP32 1e-5 relative (vs FP64).
"""
import numpy as np
import pytest

import synth
from tests._common import OracleProblem, match_by_coords, rel_err, parity_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402

NRHS = 16


def _problem(shapes_orders, dtype=P.F64, seed=0, kind=P.DIFFUSION):
    ops64, ops, xs, ys, spaces = [], [], [], [], []
    for i, (shape, p) in enumerate(shapes_orders):
        mesh = synth.hex_lattice(shape, 0.05, seed=seed + i, rotate_seed=seed + 100 + i)
        S = P.Space(P.Mesh.from_dict(mesh), p, renumber=bool(i % 2))
        qd = S.qdata(kind)
        op64 = P.Operator(S, kind, qd)
        ops64.append(op64)
        if dtype == P.F64:
            ops.append(op64)
        else:
            ops.append(P.Operator(S, kind, P.lowered_qdata(qd, dtype), qdata_dtype=dtype))
        g = torch.Generator(device="cuda")
        g.manual_seed(1000 + i)
        x = torch.randn(S.ndofs, NRHS, dtype=torch.float64, device="cuda", generator=g)
        xs.append(x if dtype == P.F64 else x.float())
        ys.append(torch.empty_like(xs[-1]))
        spaces.append((mesh, S))
    return ops64, ops, xs, ys, spaces


SHAPES = [((3, 3, 2), 2), ((2, 2, 2), 6), ((4, 3, 3), 3), ((2, 2, 3), 5), ((3, 2, 2), 4),
          ((5, 4, 3), 2), ((2, 3, 2), 3), ((6, 5, 4), 1)]


def _single_columns(op64, x):
    cols = []
    for r in range(NRHS):
        cols.append(op64.apply(x[:, r].contiguous().double()))
    return torch.stack(cols, dim=1)


@pytest.mark.parametrize("dtype,tol", [(P.F64, 1e-12), (P.F32, 1e-5)])
def test_batch_columns_match_single_applies(dtype, tol):
    ops64, ops, xs, ys, _ = _problem(SHAPES, dtype)
    B = P.Batch(ops, NRHS)
    B.apply(xs, ys)
    torch.cuda.synchronize()
    for op64, x, y in zip(ops64, xs, ys):
        ref = _single_columns(op64, x)
        err = parity_err(y.double().cpu().numpy(), ref.cpu().numpy())
        assert err <= tol, err


def test_every_tile_candidate_agrees():
    ops64, ops, xs, ys, _ = _problem(SHAPES[:5])
    B = P.Batch(ops, NRHS)
    B.apply(xs, ys)
    ref = [y.clone() for y in ys]
    orders = sorted({o.space.p for o in ops})
    for cand in range(6):
        for p in orders:
            try:
                B.set_tile(p, cand)
            except P.PafemError:
                B.set_tile(p, -1)
        B.apply(xs, ys)
        for a, b in zip(ys, ref):
            assert float((a - b).norm() / b.norm()) <= 1e-13


MFMA = 5  # the FP64 matrix-core candidate (orders 1..4, 16 right-hand sides per workgroup)


@pytest.mark.parametrize("kind", [P.DIFFUSION, P.MASS])
def test_matrix_core_candidate_matches_single_applies(kind):
    """Every column of the matrix-core batch against the single FP64 apply of its mesh,
    orders 1..4, several element counts, constrained operators."""
    shapes = [s for s in SHAPES if s[1] <= 4]
    ops64, ops, xs, ys, _ = _problem(shapes, seed=3, kind=kind)
    B = P.Batch(ops, NRHS)
    for p in sorted({o.space.p for o in ops}):
        B.set_tile(p, MFMA)
    assert all(t["candidate"] == MFMA for t in B.describe()["groups"])
    B.apply(xs, ys)
    torch.cuda.synchronize()
    for op64, x, y in zip(ops64, xs, ys):
        ref = _single_columns(op64, x)
        err = parity_err(y.cpu().numpy(), ref.cpu().numpy())
        assert err <= 1e-12, (op64.space.p, err)


def test_matrix_core_candidate_refused_where_not_built():
    ops64, ops, xs, ys, _ = _problem([((2, 2, 2), 5)])
    B = P.Batch(ops, NRHS)
    with pytest.raises(P.PafemError):
        B.set_tile(5, MFMA)
    ops64, ops, xs, ys, _ = _problem([((2, 2, 2), 3)], dtype=P.F32)
    B = P.Batch(ops, NRHS)
    with pytest.raises(P.PafemError):
        B.set_tile(3, MFMA)


def test_graph_replays_match_eager(tmp_path):
    ops64, ops, xs, ys, _ = _problem(SHAPES[:4], seed=7)
    B = P.Batch(ops, NRHS)
    B.autotune(xs, ys, cache_path=str(tmp_path / "tiles.txt"), reps=2)
    desc = B.describe()
    assert len(desc["tuning"]) > 0 and (tmp_path / "tiles.txt").exists()
    refs = [_single_columns(o, x) for o, x in zip(ops64, xs)]
    for rep in range(4):
        B.apply(xs, ys)
        torch.cuda.synchronize()
        for y, ref in zip(ys, refs):
            assert float((y - ref).norm() / ref.norm()) <= 1e-12
        # unrelated eager work between replays
        for x in xs:
            x.mul_(1.0)
        _ = [o.apply(x[:, 0].contiguous()) for o, x in zip(ops64, xs)]
    # a second batch reads the cache instead of timing
    B2 = P.Batch(ops, NRHS)
    B2.autotune(xs, ys, cache_path=str(tmp_path / "tiles.txt"), reps=2)
    assert B2.describe()["tuning"] == []


def test_batch_against_oracle():
    """Inputs from position-keyed random values on each side's own dof coordinates."""
    cases = [((3, 2, 2), 3), ((2, 2, 2), 2)]
    ops, xs, ys, refs = [], [], [], []
    for i, (shape, p) in enumerate(cases):
        mesh = synth.hex_lattice(shape, 0.05, seed=30 + i, rotate_seed=40 + i)
        S = P.Space(P.Mesh.from_dict(mesh), p)
        ops.append(P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION)))
        X = S.dof_coords()
        xs.append(torch.as_tensor(np.stack([synth.hash_normal(X, seed=r) for r in range(NRHS)], 1),
                                  device="cuda").contiguous())
        ys.append(torch.empty_like(xs[-1]))
        refs.append((OracleProblem(mesh, p), X))
    B = P.Batch(ops, NRHS)
    B.apply(xs, ys)
    for (ref, X), y in zip(refs, ys):
        Xo = np.stack([synth.hash_normal(ref.coords, seed=r) for r in range(NRHS)], 1)
        perm = match_by_coords(X, ref.coords)
        assert parity_err(y.cpu().numpy(), (ref.Kc @ Xo)[perm]) <= 1e-12
