"""Parity at the scale-sweep sizes: ~1e7 dofs per order p = 1..8 on the benchmark's
lattices (5% jitter, lognormal coefficient per quadrature point), in the launch
configuration the benchmark times (constrained operator, atomic scatter).

The oracle cannot assemble 1e7-dof matrices, so it recomputes sampled outputs one
by one: for a few centre elements (random ones and two corners) it assembles the
3x3x3 block of elements around the centre from scratch.  Every element that
touches a dof of the centre element lies in that block, so the block's
(unconstrained) rows of those dofs are complete.  The essential set comes from
the node positions (dofs on the cube's faces), independent of the library:
y_b = x_b there, and free rows ignore essential columns (symmetric elimination).
Inputs are position-keyed on both sides; results are matched by node position.
Bar: essential outputs exact; free outputs within 1e-12 relative (2-norm over the
sampled free dofs, which are measured apart: their values are O(h) (diffusion) and
O(h^3) (mass) smaller than the O(1) essential ones).
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import synth
from tests._common import on_boundary, patch_rows, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402

TARGET_DOFS = 1e7
TOL = 1e-12


def _lattice_n(p):
    return max(1, int(round((TARGET_DOFS ** (1.0 / 3.0) - 1.0) / p)))


@pytest.mark.parametrize("p", range(1, 9))
def test_bench_size_applies_on_sampled_rows(p):
    n = _lattice_n(p)
    mesh = synth.hex_lattice(n, 0.05, seed=2)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=3)
    S = P.Space(P.Mesh.from_dict(mesh), p)
    assert 0.9e7 < S.ndofs < 1.1e7
    Xlib = S.dof_coords()
    seed = 50 + p
    x = torch.as_tensor(synth.hash_normal(Xlib, seed=seed), device="cuda")
    kc = torch.as_tensor(kappa, device="cuda")
    rng = np.random.default_rng(60 + p)
    centres = [0, E - 1] + [int(c) for c in rng.integers(0, E, size=6)]
    print(f"p={p}: n={n}, {E} elements, {S.ndofs} dofs", flush=True)
    picks = {}
    for kind in (P.DIFFUSION, P.MASS):
        op = P.Operator(S, kind, S.qdata(kind, coeff=kc))
        y = op.apply(x).cpu().numpy()
        got, want, ess = [], [], []
        for c in centres:
            yo, Xo = patch_rows(mesh, kappa, p, c, "diffusion" if kind == P.DIFFUSION else "mass",
                                seed)
            if c not in picks:
                # library dofs near the centre element, matched by position
                lo, hi = Xo.min(axis=0) - 1e-9, Xo.max(axis=0) + 1e-9
                cand = np.flatnonzero(np.all((Xlib >= lo) & (Xlib <= hi), axis=1))
                dist, idx = cKDTree(Xlib[cand]).query(Xo)
                assert dist.max() < 1e-10, "node positions do not match"
                picks[c] = cand[idx]
            got.append(y[picks[c]])
            want.append(yo)
            ess.append(on_boundary(Xo))
        got, want, ess = np.concatenate(got), np.concatenate(want), np.concatenate(ess)
        err = rel_err(got[~ess], want[~ess])
        name = "diffusion" if kind == P.DIFFUSION else "mass"
        print(f"p={p} {name}: sampled {len(got)} outputs ({int(ess.sum())} essential), "
              f"free rel err {err:.2e}", flush=True)
        assert np.array_equal(got[ess], want[ess])
        assert (~ess).sum() > 0 and err <= TOL
        del op


def _sample(Xlib, y, mesh, kappa, p, centres, kind, seed, picks):
    got, want, ess = [], [], []
    for c in centres:
        yo, Xo = patch_rows(mesh, kappa, p, c, kind, seed)
        if c not in picks:
            lo, hi = Xo.min(axis=0) - 1e-9, Xo.max(axis=0) + 1e-9
            cand = np.flatnonzero(np.all((Xlib >= lo) & (Xlib <= hi), axis=1))
            dist, idx = cKDTree(Xlib[cand]).query(Xo)
            assert dist.max() < 1e-10, "node positions do not match"
            picks[c] = cand[idx]
        got.append(y[picks[c]])
        want.append(yo)
        ess.append(on_boundary(Xo))
    return np.concatenate(got), np.concatenate(want), np.concatenate(ess)


def test_mixed_precision_config_applies_on_sampled_rows():
    """The refinement benchmark's mesh: quadratic geometry warped by 0.05 sin sin sin,
    45^3 elements, p = 6 (19.9M dofs), coefficient 1.  The FP64, FP32 and BF16-D applies
    against the oracle's rows (bars as at small size: 1e-12, 1e-5, 1e-2)."""
    p, n = 6, 45
    mesh = synth.q2_warped_lattice(n, 0.05)
    E = mesh["hex"].shape[0]
    S = P.Space(P.Mesh.from_dict(mesh), p)
    Xlib = S.dof_coords()
    seed = 71
    x = torch.as_tensor(synth.hash_normal(Xlib, seed=seed), device="cuda")
    qd = S.qdata(P.DIFFUSION)
    rng = np.random.default_rng(72)
    centres = [0, E - 1] + [int(c) for c in rng.integers(0, E, size=4)]
    print(f"mixed config: {E} elements, {S.ndofs} dofs", flush=True)
    picks = {}
    for name, dt, tol in (("f64", P.F64, 1e-12), ("f32", P.F32, 1e-5), ("bf16", P.BF16, 1e-2)):
        if dt == P.F64:
            op = P.Operator(S, P.DIFFUSION, qd)
            y = op.apply(x)
        else:
            op = P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, dt), qdata_dtype=dt)
            y = op.apply(x.float())
        got, want, ess = _sample(Xlib, y.double().cpu().numpy(), mesh, None, p, centres,
                                 "diffusion", seed, picks)
        err = rel_err(got[~ess], want[~ess])
        print(f"mixed config {name}: {len(got)} sampled outputs, free rel err {err:.2e}", flush=True)
        assert err <= tol
        ess_tol = 0.0 if dt == P.F64 else 1e-7
        assert np.all(np.abs(got[ess] - want[ess]) <= ess_tol * np.abs(want[ess]))
        del op, y


def test_batched_config_columns_match_single_applies():
    """The batched benchmark's 32 uneven meshes (1e4..1e6 dofs, p = 2..6) with 16
    right-hand sides each, in one batch launch: every column equals the single-vector
    FP64 apply of its mesh (FP64 batch to 1e-12, FP32 batch to 1e-5)."""
    nrhs = 16
    specs = synth.uneven_mesh_list(32)
    spaces, qds = [], []
    for sp in specs:
        S = P.Space(P.Mesh.from_dict(synth.hex_lattice(sp["n"], 0.05, seed=sp["mesh_seed"])), sp["p"])
        spaces.append(S)
        qds.append(S.qdata(P.DIFFUSION))
    for dt, tol in ((P.F64, 1e-12), (P.F32, 1e-5)):
        ops, xs, ys, ops64 = [], [], [], []
        for i, (S, qd) in enumerate(zip(spaces, qds)):
            ops64.append(P.Operator(S, P.DIFFUSION, qd))
            if dt == P.F64:
                ops.append(ops64[-1])
            else:
                ops.append(P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, dt), qdata_dtype=dt))
            g = torch.Generator(device="cuda")
            g.manual_seed(5000 + i)
            x = torch.randn(S.ndofs, nrhs, dtype=torch.float64, device="cuda", generator=g)
            xs.append(x if dt == P.F64 else x.float())
            ys.append(torch.empty_like(xs[-1]))
        B = P.Batch(ops, nrhs)
        B.apply(xs, ys)
        worst = 0.0
        for op64, x, y in zip(ops64, xs, ys):
            for r in range(nrhs):
                ref = op64.apply(x[:, r].double().contiguous())
                worst = max(worst, float((y[:, r].double() - ref).norm() / ref.norm()))
        print(f"batched config {'f64' if dt == P.F64 else 'f32'}: worst column rel err {worst:.2e}",
              flush=True)
        assert worst <= tol
        del B


def _element_prolongation(mesh, pc, pf, c, seed):
    """Oracle prolongation restricted to element c alone: the coarse function built
    from position-keyed values at c's coarse nodes (0 on the cube's faces), evaluated
    at c's fine nodes (0 on the cube's faces), and those fine nodes' coordinates."""
    from oracle import pmg
    sub = synth.sub_mesh(mesh, [c])
    Pl = pmg.interpolation(sub, pc, pf, free_only=False)
    Xc = oracle.H1Space(sub, pc).dof_coordinates()
    Xf = oracle.H1Space(sub, pf).dof_coordinates()
    xc = np.where(on_boundary(Xc), 0.0, synth.hash_normal(Xc, seed=seed))
    y = Pl @ xc
    return np.where(on_boundary(Xf), 0.0, y), Xf


@pytest.mark.parametrize("pf", [3, 6])
def test_order_multigrid_at_bench_size(pf):
    """The multigrid benchmark's problems (~1e7 dofs, orders pf -> pf/2 -> ... -> 1):
    prolongation on sampled elements against the oracle's element-local definition
    (1e-12); restriction is its adjoint, <P a, b> = <a, P^T b> (1e-12); a V-cycle
    without coarse iterations (a linear map) is symmetric (1e-10); flexible CG with
    the V-cycle reaches the Jacobi-PCG solution."""
    n = _lattice_n(pf)
    mesh = synth.hex_lattice(n, 0.05, seed=2)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, pf + 2, 1.0, seed=3)
    kc = torch.as_tensor(kappa.reshape(-1), device="cuda")
    M = P.Mesh.from_dict(mesh)
    orders = [pf]
    while orders[-1] > 1:
        orders.append(orders[-1] // 2)
    spaces = [P.Space(M, q) for q in orders]
    print(f"multigrid p={pf}: orders {orders}, dofs {[S.ndofs for S in spaces]}", flush=True)
    # prolongation on sampled elements
    Sf, Sc = spaces[0], spaces[1]
    Xf, Xc = Sf.dof_coords(), Sc.dof_coords()
    y = P.prolongate(Sc, Sf, torch.as_tensor(synth.hash_normal(Xc, seed=5), device="cuda"))
    y = y.cpu().numpy()
    rng = np.random.default_rng(8)
    got, want = [], []
    for c in [0, E - 1] + [int(v) for v in rng.integers(0, E, size=6)]:
        yo, Xo = _element_prolongation(mesh, orders[1], pf, c, 5)
        lo_, hi_ = Xo.min(axis=0) - 1e-9, Xo.max(axis=0) + 1e-9
        cand = np.flatnonzero(np.all((Xf >= lo_) & (Xf <= hi_), axis=1))
        dist, idx = cKDTree(Xf[cand]).query(Xo)
        assert dist.max() < 1e-10
        got.append(y[cand[idx]])
        want.append(yo)
    err = rel_err(np.concatenate(got), np.concatenate(want))
    print(f"multigrid p={pf}: sampled prolongation rel err {err:.2e}", flush=True)
    assert err <= 1e-12
    # restriction is the adjoint of prolongation
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    a = torch.randn(Sc.ndofs, dtype=torch.float64, device="cuda", generator=g)
    bf = torch.randn(Sf.ndofs, dtype=torch.float64, device="cuda", generator=g)
    lhs = float(torch.dot(P.prolongate(Sc, Sf, a), bf))
    rhs = float(torch.dot(a, P.restrict(Sf, Sc, bf)))
    print(f"multigrid p={pf}: <Pa,b> {lhs:.15e} <a,P^T b> {rhs:.15e}", flush=True)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))
    # hierarchy
    ops, diags, lmax = [], [], []
    for l, S in enumerate(spaces):
        c = kc if l == 0 else S.coeff_mean(kc, q1d_in=pf + 2, q1d_out=S.p + 2)
        ops.append(P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION, coeff=c)))
        diags.append(ops[-1].diagonal())
        v = torch.randn(S.ndofs, dtype=torch.float64, device="cuda", generator=g)
        lmax.append(ops[-1].lambda_max(diags[-1], v, 20))
    lin = P.PMG(ops, diags, lmax, degree=2, coarse_iters=0)
    u = torch.randn(Sf.ndofs, dtype=torch.float64, device="cuda", generator=g)
    w = torch.randn(Sf.ndofs, dtype=torch.float64, device="cuda", generator=g)
    s1, s2 = float(torch.dot(lin.vcycle(u), w)), float(torch.dot(u, lin.vcycle(w)))
    print(f"multigrid p={pf}: <V u, w> {s1:.15e} <u, V w> {s2:.15e}", flush=True)
    assert abs(s1 - s2) <= 1e-10 * (abs(s1) + abs(s2))
    del lin
    G = P.PMG(ops, diags, lmax, degree=2, coarse_iters=10)
    b = Sf.linear_form(P.SOURCE_SINE)
    x, info = G.fcg(b, rel_tol=1e-8, max_iter=300, history=False)
    xj, ij = ops[0].pcg(b, diag=diags[0], rel_tol=1e-8, max_iter=20000, history=False)
    diff = float((x - xj).norm() / xj.norm())
    print(f"multigrid p={pf}: fcg {info['iters']} its (true rel res {info['true_rel_res']:.2e}), "
          f"jacobi {ij['iters']} its, solutions differ by {diff:.2e}", flush=True)
    assert info["converged"] and info["true_rel_res"] <= 1.5e-8
    assert diff <= 1e-6
