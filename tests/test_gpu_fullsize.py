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
from tests._common import on_boundary, patch_rows, rel_err, parity_err

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
        err = parity_err(got[~ess], want[~ess])
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
        err = parity_err(got[~ess], want[~ess])
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
                worst = max(worst, parity_err(y[:, r].double().cpu().numpy(), ref.cpu().numpy()))
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
    err = parity_err(np.concatenate(got), np.concatenate(want))
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


@pytest.mark.parametrize("p", [1, 3, 6, 8])
def test_bench_size_integrator_properties(p):
    """The further integrators at the sweep sizes, in the configuration the benchmark
    times, through identities that hold exactly (up to rounding) at any size.  With the
    linear field u_c = sum_d A[c, d] x_d + b_c (in the space): divergence sum_c V_c u_c =
    tr(A) M_kappa 1; gradient of u_0, component c: A[0, c] M_kappa 1; convection of u_0
    with constant beta: (beta . A[0]) M_1 1.  Elasticity annihilates the six rigid-body
    fields, and its constrained form returns x on the essential dofs."""
    n = _lattice_n(p)
    mesh = synth.hex_lattice(n, 0.05, seed=2)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=3)
    S = P.Space(P.Mesh.from_dict(mesh), p)
    del mesh
    X = S.dof_coords()
    kc = torch.as_tensor(kappa, device="cuda")
    N = S.ndofs
    print(f"p={p}: {E} elements, {N} dofs", flush=True)
    A = np.array([[0.3, -1.1, 0.4], [0.9, 1.7, -0.2], [0.5, 0.8, -2.3]])
    u = X @ A.T + np.array([0.2, -0.7, 1.3])          # u_c = sum_d A[c, d] x_d + b_c
    ones = torch.ones(N, dtype=torch.float64, device="cuda")
    mk1 = P.Operator(S, P.MASS, S.qdata(P.MASS, coeff=kc), constrained=False).apply(ones)
    mk1 = mk1.cpu().numpy()
    u3 = torch.as_tensor(np.ascontiguousarray(u.T).ravel(), device="cuda")
    # divergence: div u = tr(A)
    qg = S.qdata(P.DIVERGENCE, coeff=kc)
    y = P.Operator(S, P.DIVERGENCE, qg, constrained=False).apply(u3).cpu().numpy()
    err = parity_err(y, np.trace(A) * mk1)
    print(f"p={p} divergence: rel err {err:.2e}", flush=True)
    assert err <= TOL
    # gradient of the scalar u_0 = A[0] . x + b_0: component c is A[0, c] M_kappa 1
    y = P.Operator(S, P.GRADIENT, qg, constrained=False).apply(u3[:N].contiguous())
    y = y.cpu().numpy().reshape(3, -1)
    err = max(parity_err(y[c], A[0, c] * mk1) for c in range(3))
    print(f"p={p} gradient: rel err {err:.2e}", flush=True)
    assert err <= TOL
    del qg
    # convection of u_0 with constant beta: beta . grad u_0 = beta . A[0]
    beta = np.array([1.0, 0.5, 0.25])
    bq = torch.tensor(beta, dtype=torch.float64, device="cuda").repeat(E * (p + 2) ** 3)
    conv = P.Operator(S, P.CONVECTION, S.qdata(P.CONVECTION, coeff=bq), constrained=False)
    del bq
    m1 = P.Operator(S, P.MASS, S.qdata(P.MASS), constrained=False).apply(ones).cpu().numpy()
    y = conv.apply(u3[:N].contiguous()).cpu().numpy()
    err = parity_err(y, float(beta @ A[0]) * m1)
    print(f"p={p} convection: rel err {err:.2e}", flush=True)
    assert err <= TOL
    del conv
    # elasticity: rigid-body fields, and the constrained form's essential rows
    lm = torch.stack([kc, 0.5 * kc], dim=-1).contiguous()
    qe = S.qdata(P.ELASTICITY, coeff=lm)
    del lm
    el = P.Operator(S, P.ELASTICITY, qe, constrained=False)
    w = torch.as_tensor(np.concatenate([synth.hash_normal(X, seed=70 + c) for c in range(3)]),
                        device="cuda")
    scale = float(el.apply(w).abs().max())
    worst = 0.0
    modes = [np.tile(e_, (N, 1)) for e_ in np.eye(3)] + [np.cross(v, X) for v in np.eye(3)]
    for m in modes:
        r = el.apply(torch.as_tensor(np.ascontiguousarray(m.T).ravel(), device="cuda"))
        worst = max(worst, float(r.abs().max()) / scale)
    print(f"p={p} elasticity: rigid-body residual {worst:.2e} of max|K w|", flush=True)
    assert worst <= 1e-12
    elc = P.Operator(S, P.ELASTICITY, qe, constrained=True)
    yc = elc.apply(w).cpu().numpy().reshape(3, -1)
    bd = S.boundary_dofs()
    wn = w.cpu().numpy().reshape(3, -1)
    assert np.array_equal(yc[:, bd], wn[:, bd])


@pytest.mark.parametrize("p", range(1, 9))
def test_bench_size_diffusion_mass_identities(p):
    """The stored-D diffusion and mass applies at the sweep sizes (~1e7 dofs, lognormal
    kappa = rho per quadrature point), over every element, through identities that hold
    exactly (up to rounding) at any size.  x_a are the coordinate fields, which the
    space holds exactly (trilinear geometry), so grad x_a = e_a at every point:
      * K_kappa 1 = 0, entry by entry (unconstrained);
      * x_a^T K_kappa x_b = delta_ab 1^T M_kappa 1;
      * K_1 (c . x + c0) = 0 on every row whose node is off the boundary (kappa = 1:
        the element integrals of grad phi_i . c are exact at p + 2 Gauss points on
        trilinear hexes, and their sum is the flux of c through the boundary);
      * 1^T M_1 1 = |unit cube| = 1, x_a^T M_1 1 = 1/2, x_a^T M_1 x_b = 1/4 or 1/3
        (exact at p + 2 Gauss points);
      * M_kappa 1 = component 0 of the gradient operator on x_0 and, for p >= 2,
        M_kappa x_0 = component 0 of the gradient operator on x_0^2 / 2 (held
        exactly for p >= 2), entry by entry;
      * the constrained operators (the benchmark's launch): w^T A v = v^T A w,
        y_b = x_b on the essential dofs and the free rows equal the unconstrained
        operator applied to x with its essential entries set to 0."""
    n = _lattice_n(p)
    mesh = synth.hex_lattice(n, 0.05, seed=2)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=3)
    S = P.Space(P.Mesh.from_dict(mesh), p)
    del mesh
    X = S.dof_coords()
    N = S.ndofs
    print(f"p={p}: {E} elements, {N} dofs", flush=True)
    kc = torch.as_tensor(kappa, device="cuda")
    del kappa
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    ones = torch.ones(N, dtype=torch.float64, device="cuda")
    xa = [dev(X[:, a]) for a in range(3)]
    w = dev(synth.hash_normal(X, seed=90 + p))
    v = dev(synth.hash_normal(X, seed=91 + p))
    ess = on_boundary(X)
    ess_t = torch.as_tensor(ess, device="cuda")

    def dot(a, b):
        return float(torch.dot(a, b))

    # diffusion with the lognormal coefficient
    qk = S.qdata(P.DIFFUSION, coeff=kc)
    Ku = P.Operator(S, P.DIFFUSION, qk, constrained=False)
    scale = float(Ku.apply(w).abs().max())
    r = float(Ku.apply(ones).abs().max()) / scale
    print(f"p={p} diffusion: max|K 1| {r:.2e} of max|K w|", flush=True)
    assert r <= TOL
    qm = S.qdata(P.MASS, coeff=kc)
    vol_k = dot(ones, P.Operator(S, P.MASS, qm, constrained=False).apply(ones))
    Kx = [Ku.apply(xa[b]) for b in range(3)]
    worst = max(abs(dot(xa[a], Kx[b]) - (vol_k if a == b else 0.0)) / vol_k
                for a in range(3) for b in range(3))
    print(f"p={p} diffusion: x_a^T K x_b vs delta_ab 1^T M 1 = {vol_k:.12f}: {worst:.2e}",
          flush=True)
    assert worst <= TOL
    del Kx
    # constrained forms (as benchmarked)
    for kind, qd in ((P.DIFFUSION, qk), (P.MASS, qm)):
        name = "diffusion" if kind == P.DIFFUSION else "mass"
        Ac = P.Operator(S, kind, qd)
        Au = P.Operator(S, kind, qd, constrained=False)
        Av, Aw = Ac.apply(v), Ac.apply(w)
        s1, s2 = dot(w, Av), dot(v, Aw)
        sym = abs(s1 - s2) / (float(w.norm() * Av.norm()) + float(v.norm() * Aw.norm()))
        yb = Aw.cpu().numpy()
        wn = w.cpu().numpy()
        assert np.array_equal(yb[ess], wn[ess])
        y0 = Au.apply(torch.where(ess_t, torch.zeros_like(w), w)).cpu().numpy()
        free = parity_err(yb[~ess], y0[~ess])
        print(f"p={p} {name} constrained: symmetry {sym:.2e}, free rows vs unconstrained "
              f"{free:.2e}", flush=True)
        assert sym <= TOL and free <= TOL
        del Ac, Au, Av, Aw
    del Ku, qk
    # diffusion with kappa = 1 on a linear field: interior rows vanish
    K1 = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION), constrained=False)
    c = np.array([0.7, -1.3, 0.4])
    y = K1.apply(dev(X @ c + 0.25)).cpu().numpy()
    scale = float(K1.apply(w).abs().max())
    r = np.abs(y[~ess]).max() / scale
    print(f"p={p} diffusion kappa=1: max interior |K (c.x + c0)| {r:.2e} of max|K w|", flush=True)
    assert r <= TOL
    del K1
    # mass with rho = 1: moments of the unit cube
    M1 = P.Operator(S, P.MASS, S.qdata(P.MASS), constrained=False)
    m1 = M1.apply(ones)
    got = [dot(ones, m1)] + [dot(xa[a], m1) for a in range(3)]
    want = [1.0, 0.5, 0.5, 0.5]
    Mx = [M1.apply(xa[b]) for b in range(3)]
    for a in range(3):
        for b in range(3):
            got.append(dot(xa[a], Mx[b]))
            want.append(1.0 / 3.0 if a == b else 0.25)
    worst = max(abs(g - t) / t for g, t in zip(got, want))
    print(f"p={p} mass rho=1: moments of the unit cube, worst rel err {worst:.2e}", flush=True)
    assert worst <= TOL
    del M1, Mx, m1
    # mass with the lognormal coefficient against the gradient operator, every row
    Mk = P.Operator(S, P.MASS, qm, constrained=False)
    qg = S.qdata(P.DIVERGENCE, coeff=kc)
    G = P.Operator(S, P.GRADIENT, qg, constrained=False)
    g0 = G.apply(xa[0]).view(3, -1)
    err = parity_err(g0[0].cpu().numpy(), Mk.apply(ones).cpu().numpy())
    rest = float(g0[1:].abs().max()) / float(g0[0].abs().max())
    print(f"p={p} mass kappa: M 1 vs gradient of x_0 {err:.2e} (other components {rest:.2e})",
          flush=True)
    assert err <= TOL and rest <= TOL
    if p >= 2:
        g2 = G.apply(0.5 * xa[0] * xa[0]).view(3, -1)
        err = parity_err(g2[0].cpu().numpy(), Mk.apply(xa[0]).cpu().numpy())
        print(f"p={p} mass kappa: M x_0 vs gradient of x_0^2/2 {err:.2e}", flush=True)
        assert err <= TOL
