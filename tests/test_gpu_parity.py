"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

Inputs are seeded synthetic meshes; input vectors are pseudo-random values keyed
by dof position (``synth.hash_normal``), so each side evaluates them on its own
dof coordinates and no input crosses from the GPU path to the oracle.  Results
are compared after matching dofs by position.  Bar for applies, diagonals and
load vectors in FP64: ||got - want|| <= 1e-12 ||want|| and, entry by entry,
max|got - want| <= 1e-12 max|want|.
"""
import numpy as np
import pytest

import oracle
from oracle import forms
import synth
from tests._common import OracleProblem, match_by_coords, rel_err, parity_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402  (must load: no fallback)

TOL = 1e-12

# per order: lattice shape spanning several element tiles with a ragged last tile
SHAPES = {1: (5, 5, 5), 2: (5, 4, 3), 3: (4, 4, 4), 4: (3, 3, 3), 5: (3, 3, 2),
          6: (3, 2, 2), 7: (2, 2, 2), 8: (3, 1, 1)}


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _setup(mesh, p, coeff=None, renumber=False):
    S = P.Space(P.Mesh.from_dict(mesh), p, renumber=renumber)
    c = None if coeff is None else _cuda(coeff)
    return S, S.dof_coords(), c


@pytest.mark.parametrize("scatter", ["atomic", "evec"])
@pytest.mark.parametrize("p", range(1, 9))
def test_diffusion_apply(p, scatter):
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=p, rotate_seed=100 + p)
    kappa = synth.lognormal_iid(mesh["hex"].shape[0], p + 2, 1.0, seed=7)
    S, X, kc = _setup(mesh, p, kappa, renumber=(p % 2 == 0))
    op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION, coeff=kc), scatter=scatter)
    y = op.apply(_cuda(synth.hash_normal(X, seed=p))).cpu().numpy()
    ref = OracleProblem(mesh, p, coeff=kappa)
    y_ref = ref.Kc @ synth.hash_normal(ref.coords, seed=p)
    perm = match_by_coords(X, ref.coords)
    err = parity_err(y, y_ref[perm])
    print(f"diffusion p={p} {scatter}: rel err {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("p", range(1, 9))
def test_mass_apply(p):
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=20 + p)
    rho = synth.lognormal_iid(mesh["hex"].shape[0], p + 2, 1.0, seed=8)
    S, X, rc = _setup(mesh, p, rho)
    for scatter in ("atomic", "evec"):
        op = P.Operator(S, P.MASS, S.qdata(P.MASS, coeff=rc), scatter=scatter)
        y = op.apply(_cuda(synth.hash_normal(X, seed=3))).cpu().numpy()
        ref = OracleProblem(mesh, p, rho=rho)
        y_ref = ref.Mc @ synth.hash_normal(ref.coords, seed=3)
        perm = match_by_coords(X, ref.coords)
        assert parity_err(y, y_ref[perm]) <= TOL


@pytest.mark.parametrize("kind", [P.DIFFUSION, P.MASS])
@pytest.mark.parametrize("p,shape", [(1, (2, 2, 2)), (2, (2, 2, 1)), (3, (2, 1, 1)), (5, (1, 1, 1))])
def test_brute_force_columns(kind, p, shape):
    """A e_j for every unit vector rebuilds the oracle's assembled constrained matrix."""
    mesh = synth.hex_lattice(shape, 0.15, seed=5, rotate_seed=6)
    S, X, _ = _setup(mesh, p)
    op = P.Operator(S, kind, S.qdata(kind))
    n = S.ndofs
    A = np.empty((n, n))
    e = torch.zeros(n, dtype=torch.float64, device="cuda")
    for j in range(n):
        e.zero_()
        e[j] = 1.0
        A[:, j] = op.apply(e).cpu().numpy()
    ref = OracleProblem(mesh, p)
    Aref = (ref.Kc if kind == P.DIFFUSION else ref.Mc).toarray()
    perm = match_by_coords(X, ref.coords)
    Aref = Aref[np.ix_(perm, perm)]
    assert np.abs(A - Aref).max() <= TOL * np.abs(Aref).max()
    assert np.abs(A - A.T).max() <= TOL * np.abs(A).max()


@pytest.mark.parametrize("p", [2, 3, 6])
def test_quadratic_geometry(p):
    mesh = synth.q2_warped_lattice(2, 0.05)
    S, X, _ = _setup(mesh, p)
    op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION))
    y = op.apply(_cuda(synth.hash_normal(X, seed=11))).cpu().numpy()
    ref = OracleProblem(mesh, p)
    perm = match_by_coords(X, ref.coords)
    assert parity_err(y, (ref.Kc @ synth.hash_normal(ref.coords, seed=11))[perm]) <= TOL


@pytest.mark.parametrize("p", range(1, 9))
def test_diagonal(p):
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=30 + p, rotate_seed=31)
    kappa = synth.lognormal_iid(mesh["hex"].shape[0], p + 2, 1.0, seed=9)
    S, X, kc = _setup(mesh, p, kappa)
    ref = OracleProblem(mesh, p, coeff=kappa, rho=kappa)
    perm = match_by_coords(X, ref.coords)
    for kind, A in ((P.DIFFUSION, ref.Kc), (P.MASS, ref.Mc)):
        op = P.Operator(S, kind, S.qdata(kind, coeff=kc))
        d = op.diagonal().cpu().numpy()
        assert parity_err(d, A.diagonal()[perm]) <= TOL


@pytest.mark.parametrize("p", range(1, 9))
def test_linear_form(p):
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=40 + p)
    S, X, _ = _setup(mesh, p)
    ref = OracleProblem(mesh, p)
    perm = match_by_coords(X, ref.coords)
    b = S.linear_form(P.SOURCE_SINE).cpu().numpy()
    assert parity_err(b, ref.load(synth.sine_source)[perm]) <= TOL
    b1 = S.linear_form(P.SOURCE_CONST, scale=2.5).cpu().numpy()
    assert parity_err(b1, ref.load(lambda x: np.full(x.shape[:-1], 2.5))[perm]) <= TOL
    fq = synth.lognormal_iid(mesh["hex"].shape[0], p + 2, 0.5, seed=12)
    b2 = S.linear_form(P.SOURCE_ARRAY, f_qp=_cuda(fq)).cpu().numpy()
    assert parity_err(b2, ref.load(fq)[perm]) <= TOL


def test_unconstrained_invariants():
    """Without BC: 1^T M 1 = volume = 1 and the diffusion operator annihilates constants."""
    mesh = synth.hex_lattice(4, 0.1, seed=2)
    S, X, _ = _setup(mesh, 3)
    one = torch.ones(S.ndofs, dtype=torch.float64, device="cuda")
    M = P.Operator(S, P.MASS, S.qdata(P.MASS), constrained=False)
    K = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION), constrained=False)
    assert abs(float(torch.dot(one, M.apply(one))) - 1.0) < 1e-13
    assert float(K.apply(one).abs().max()) < 1e-12


def test_evec_scatter_is_bitwise_reproducible():
    mesh = synth.hex_lattice(6, 0.1, seed=1)
    S, X, _ = _setup(mesh, 3)
    op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION), scatter="evec")
    x = _cuda(synth.hash_normal(X, seed=1))
    y1, y2 = op.apply(x), op.apply(x)
    assert torch.equal(y1, y2)


def test_inverted_element_rejected():
    mesh = synth.hex_lattice(2)
    h = mesh["hex"].copy()
    h[3] = h[3][[4, 5, 6, 7, 0, 1, 2, 3]]          # mirror: det J < 0 everywhere
    S = P.Space(P.Mesh(mesh["vertices"], h), 2)
    with pytest.raises(P.PafemError) as ei:
        S.qdata(P.DIFFUSION)
    assert ei.value.code == -1 and "element 3" in str(ei.value)


def test_small_poisson_solve():
    """Unit cube 8^3, 10% jitter, p = 2, f from the sine solution, Jacobi-PCG."""
    mesh = synth.hex_lattice(8, 0.1, seed=1)
    S, X, _ = _setup(mesh, 2)
    assert S.ndofs == 4913
    op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION))
    b = S.linear_form(P.SOURCE_SINE)
    x, info = op.pcg(b, rel_tol=1e-13, max_iter=2000)
    assert info["status"] == "OK" and info["converged"]
    assert info["true_rel_res"] < 1e-12
    ref = OracleProblem(mesh, 2)
    perm = match_by_coords(X, ref.coords)
    bref = ref.load(synth.sine_source)
    assert parity_err(b.cpu().numpy(), bref[perm]) <= TOL
    import scipy.sparse.linalg as spla
    xd = spla.spsolve(ref.Kc.tocsc(), bref)
    err = rel_err(x.cpu().numpy(), xd[perm])
    print(f"poisson: iters {info['iters']} solution rel err vs direct {err:.2e}")
    assert err < 1e-11
    # same iteration history as the oracle's PCG up to roundoff
    r = oracle.pcg(ref.Kc, bref, ref.Kc.diagonal(), tol=1e-13)
    assert abs(r["iters"] - info["iters"]) <= 2
    hist = info["history"]
    assert np.allclose(hist[:20], r["history"][:20], rtol=1e-8)
    assert oracle.l2_error(ref.space, x.cpu().numpy()[np.argsort(perm)], synth.sine_solution) < 1e-3


def test_pcg_from_a_guess_with_boundary_values():
    """A starting guess that is nonzero on essential dofs makes the first directions
    nonzero there: the step length must include those rows (q_b = d_b).  The
    iteration history follows the oracle's PCG from the same guess."""
    mesh = synth.hex_lattice(6, 0.1, seed=2)
    S, X, _ = _setup(mesh, 2)
    op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION))
    b = S.linear_form(P.SOURCE_SINE)
    ref = OracleProblem(mesh, 2)
    perm = match_by_coords(X, ref.coords)
    x0_or = synth.hash_normal(ref.coords, seed=31)
    x0 = torch.as_tensor(synth.hash_normal(X, seed=31), device="cuda")
    assert float(x0[torch.as_tensor(S.boundary_dofs(), device="cuda").long()].abs().max()) > 0
    x, info = op.pcg(b, x=x0.clone(), rel_tol=1e-12, max_iter=2000)
    assert info["status"] == "OK" and info["converged"]
    bref = ref.load(synth.sine_source)
    r = oracle.pcg(ref.Kc, bref, ref.Kc.diagonal(), tol=1e-12, x0=x0_or)
    print(f"guess: iters {info['iters']} oracle {r['iters']}")
    assert abs(r["iters"] - info["iters"]) <= 2
    assert np.allclose(info["history"][:20], r["history"][:20], rtol=1e-8)
    assert rel_err(x.cpu().numpy(), r["x"][perm]) < 1e-10


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_apply_on_offset_views_matches_aligned(dtype):
    """Vectors that are views at an 8-byte (f64) or 4-byte (f32) offset take the scalar
    output-init path, aligned vectors the 4-wide one; an odd dof count exercises the
    tail.  Both give the same result up to the summation order of the atomic scatter
    (which is not fixed from run to run), and nothing outside the view is written."""
    mesh = synth.hex_lattice(5, 0.1, seed=4)
    S, X, _ = _setup(mesh, 2)
    assert S.ndofs % 4 != 0
    qd = S.qdata(P.DIFFUSION)
    if dtype == "f32":
        op = P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, P.F32), qdata_dtype=P.F32)
        tdt = torch.float32
    else:
        op = P.Operator(S, P.DIFFUSION, qd)
        tdt = torch.float64
    x = torch.as_tensor(synth.hash_normal(X, seed=41), device="cuda").to(tdt)
    y = op.apply(x)
    big_x = torch.zeros(S.ndofs + 1, dtype=tdt, device="cuda")
    big_x[1:] = x
    big_y = torch.full((S.ndofs + 1,), 7.0, dtype=tdt, device="cuda")
    op.apply(big_x[1:], big_y[1:])
    tol = 1e-14 if dtype == "f64" else 1e-6
    assert float((big_y[1:] - y).norm() / y.norm()) <= tol and float(big_y[0]) == 7.0



@pytest.mark.parametrize("p", range(1, 9))
def test_diffusion_with_recomputed_geometry(p):
    """The variant that stores only w*kappa per quadrature point and rebuilds the
    trilinear Jacobian inside the apply: the oracle's operator to 1e-12 on rotated,
    jittered elements with a lognormal coefficient, in both scatter modes, and the
    stored-D apply on the same input."""
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=50 + p, rotate_seed=150 + p)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=51 + p)
    S, X, kc = _setup(mesh, p, kappa)
    qg = S.qdata(P.DIFFUSION_GEOM, coeff=kc)
    qd = S.qdata(P.DIFFUSION, coeff=kc)
    assert qg.numel() * 6 == qd.numel()
    x = _cuda(synth.hash_normal(X, seed=52 + p))
    stored = P.Operator(S, P.DIFFUSION, qd).apply(x)
    ref = OracleProblem(mesh, p, coeff=kappa)
    y_ref = ref.Kc @ synth.hash_normal(ref.coords, seed=52 + p)
    perm = match_by_coords(X, ref.coords)
    for scatter in ("atomic", "evec"):
        y = P.Operator(S, P.DIFFUSION_GEOM, qg, scatter=scatter).apply(x)
        err = parity_err(y.cpu().numpy(), y_ref[perm])
        print(f"recomputed geometry p={p} {scatter}: rel err {err:.2e}")
        assert err <= TOL
        assert float((y - stored).norm() / stored.norm()) <= TOL


def test_recomputed_geometry_limits():
    """Quadratic geometry and the diagonal are refused with an error, and so is a
    batch of such operators."""
    S2 = P.Space(P.Mesh.from_dict(synth.q2_warped_lattice(2, 0.05)), 2)
    with pytest.raises(P.PafemError):
        P.Operator(S2, P.DIFFUSION_GEOM, S2.qdata(P.DIFFUSION_GEOM))
    S1 = P.Space(P.Mesh.from_dict(synth.hex_lattice(2, 0.1, seed=1)), 2)
    op = P.Operator(S1, P.DIFFUSION_GEOM, S1.qdata(P.DIFFUSION_GEOM))
    with pytest.raises(P.PafemError):
        op.diagonal()
    with pytest.raises(P.PafemError):
        P.Batch([op], 2)


def test_pcg_with_recomputed_geometry():
    """Jacobi-PCG on the recomputed-geometry operator (diagonal taken from the
    stored-D operator) reaches the direct solution of the oracle's system, with the
    oracle PCG's iteration count."""
    mesh = synth.hex_lattice(6, 0.1, seed=3, rotate_seed=4)
    S, X, _ = _setup(mesh, 3)
    diag = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION)).diagonal()
    op = P.Operator(S, P.DIFFUSION_GEOM, S.qdata(P.DIFFUSION_GEOM))
    b = S.linear_form(P.SOURCE_SINE)
    x, info = op.pcg(b, diag=diag, rel_tol=1e-12, max_iter=2000)
    assert info["status"] == "OK" and info["converged"]
    ref = OracleProblem(mesh, 3)
    perm = match_by_coords(X, ref.coords)
    bref = ref.load(synth.sine_source)
    import scipy.sparse.linalg as spla
    xd = spla.spsolve(ref.Kc.tocsc(), bref)
    err = rel_err(x.cpu().numpy(), xd[perm])
    print(f"recomputed-geometry pcg: iters {info['iters']} rel err vs direct {err:.2e}")
    assert err < 1e-10
    r = oracle.pcg(ref.Kc, bref, ref.Kc.diagonal(), tol=1e-12)
    assert abs(r["iters"] - info["iters"]) <= 2


@pytest.mark.parametrize("p", range(1, 9))
def test_convection_apply(p):
    """int (beta . grad u) v with a seeded random velocity per quadrature point, on
    rotated jittered elements: the oracle's constrained matrix to 1e-12 in both scatter
    modes; unconstrained, constants are annihilated."""
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=60 + p, rotate_seed=160 + p)
    E = mesh["hex"].shape[0]
    Q = p + 2
    beta = np.random.default_rng(61 + p).normal(size=(E, Q ** 3, 3))
    S, X, _ = _setup(mesh, p)
    qd = S.qdata(P.CONVECTION, coeff=_cuda(beta.reshape(-1)))
    ref = oracle.H1Space(mesh, p)
    C = oracle.assemble(ref, forms.element_convection(mesh, p, Q, beta))
    Cc, _ = oracle.constrain(C, np.zeros(ref.ndofs), ref.boundary)
    perm = match_by_coords(X, ref.dof_coordinates())
    want = (Cc @ synth.hash_normal(ref.dof_coordinates(), seed=62 + p))[perm]
    x = _cuda(synth.hash_normal(X, seed=62 + p))
    for scatter in ("atomic", "evec"):
        y = P.Operator(S, P.CONVECTION, qd, scatter=scatter).apply(x).cpu().numpy()
        err = parity_err(y, want)
        print(f"convection p={p} {scatter}: rel err {err:.2e}")
        assert err <= TOL
    free = P.Operator(S, P.CONVECTION, qd, constrained=False)
    one = torch.ones(S.ndofs, dtype=torch.float64, device="cuda")
    scale = float(free.apply(x).abs().max())
    assert float(free.apply(one).abs().max()) <= 1e-12 * scale


def test_convection_limits():
    S = P.Space(P.Mesh.from_dict(synth.hex_lattice(2, 0.1, seed=1)), 2)
    beta = torch.ones(S.nelem * 64 * 3, dtype=torch.float64, device="cuda")
    qd = S.qdata(P.CONVECTION, coeff=beta)
    op = P.Operator(S, P.CONVECTION, qd)
    with pytest.raises(P.PafemError):
        op.diagonal()
    with pytest.raises(P.PafemError):
        op.pcg(torch.ones(S.ndofs, dtype=torch.float64, device="cuda"),
               diag=torch.ones(S.ndofs, dtype=torch.float64, device="cuda"))
    with pytest.raises(P.PafemError):
        P.Operator(S, P.CONVECTION, P.lowered_qdata(qd, P.F32), qdata_dtype=P.F32)
    with pytest.raises(ValueError):
        S.qdata(P.CONVECTION)


@pytest.mark.parametrize("p", range(1, 9))
def test_gradient_apply(p):
    """(grad u, v) into a vector-valued output, lognormal coefficient, rotated jittered
    elements: every component against the oracle's unconstrained matrices to 1e-12
    (p <= 4: the three-accumulator kernel; p >= 5: one pass per component)."""
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=70 + p, rotate_seed=170 + p)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=71 + p)
    S, X, kc = _setup(mesh, p, kappa, renumber=(p % 2 == 1))
    op = P.Operator(S, P.GRADIENT, S.qdata(P.GRADIENT, coeff=kc), constrained=False)
    y = op.apply(_cuda(synth.hash_normal(X, seed=72 + p))).cpu().numpy().reshape(3, -1)
    ref = oracle.H1Space(mesh, p)
    Ge = forms.element_gradient(mesh, p, p + 2, kappa)
    xo = synth.hash_normal(ref.dof_coordinates(), seed=72 + p)
    perm = match_by_coords(X, ref.dof_coordinates())
    for c in range(3):
        want = (oracle.assemble(ref, Ge[:, c]) @ xo)[perm]
        err = parity_err(y[c], want)
        print(f"gradient p={p} component {c}: rel err {err:.2e}")
        assert err <= TOL


def test_gradient_limits():
    S = P.Space(P.Mesh.from_dict(synth.hex_lattice(2, 0.1, seed=1)), 2)
    qd = S.qdata(P.GRADIENT)
    with pytest.raises(P.PafemError):
        P.Operator(S, P.GRADIENT, qd)                      # constrained is not defined
    with pytest.raises(P.PafemError):
        P.Operator(S, P.GRADIENT, qd, constrained=False, scatter="evec")
    op = P.Operator(S, P.GRADIENT, qd, constrained=False)
    with pytest.raises(P.PafemError):
        op.diagonal()
    with pytest.raises(P.PafemError):
        P.Operator(S, P.GRADIENT, P.lowered_qdata(qd, P.F32), qdata_dtype=P.F32,
                   constrained=False)


@pytest.mark.parametrize("p", range(1, 9))
def test_vector_operator_applies_per_component(p):
    """PAFEM_OP_VECTOR3: each component equals the scalar operator's apply (1e-14) and
    the oracle's constrained matrix (1e-12), for diffusion and mass."""
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=80 + p, rotate_seed=180 + p)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=81 + p)
    S, X, kc = _setup(mesh, p, kappa)
    ref = OracleProblem(mesh, p, coeff=kappa, rho=kappa)
    perm = match_by_coords(X, ref.coords)
    xs = [synth.hash_normal(X, seed=90 + c) for c in range(3)]
    xo = [synth.hash_normal(ref.coords, seed=90 + c) for c in range(3)]
    x3 = _cuda(np.concatenate(xs))
    for kind, A in ((P.DIFFUSION, ref.Kc), (P.MASS, ref.Mc)):
        qd = S.qdata(kind, coeff=kc)
        vec = P.Operator(S, kind, qd, vector=True).apply(x3).cpu().numpy().reshape(3, -1)
        sc = P.Operator(S, kind, qd)
        for c in range(3):
            ys = sc.apply(_cuda(xs[c])).cpu().numpy()
            assert parity_err(vec[c], ys) <= 1e-14
            assert parity_err(vec[c], (A @ xo[c])[perm]) <= TOL


@pytest.mark.parametrize("p", range(1, 9))
def test_divergence_apply(p):
    """(div u, q) of a three-component input, lognormal coefficient, rotated jittered
    elements: against the oracle's unconstrained matrices sum_c V_c u_c to 1e-12."""
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=100 + p, rotate_seed=200 + p)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=101 + p)
    S, X, kc = _setup(mesh, p, kappa, renumber=(p % 2 == 0))
    op = P.Operator(S, P.DIVERGENCE, S.qdata(P.DIVERGENCE, coeff=kc), constrained=False)
    x3 = _cuda(np.concatenate([synth.hash_normal(X, seed=102 + c) for c in range(3)]))
    y = op.apply(x3).cpu().numpy()
    ref = oracle.H1Space(mesh, p)
    Ve = forms.element_divergence(mesh, p, p + 2, kappa)
    Xo = ref.dof_coordinates()
    want = sum(oracle.assemble(ref, Ve[:, c]) @ synth.hash_normal(Xo, seed=102 + c)
               for c in range(3))
    err = parity_err(y, want[match_by_coords(X, Xo)])
    print(f"divergence p={p}: rel err {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("p", [2, 3, 5])
def test_divergence_properties_many_tiles(p):
    """Properties that hold at any size, on ~1e5-dof meshes: the divergence of a linear
    field A x + b is tr(A) M 1 (M the unconstrained mass operator of the same
    coefficient), and (div u, q) = -(u, grad q) for u vanishing on the boundary (unit
    coefficient; exact on trilinear elements with p + 2 points)."""
    n = {2: 24, 3: 16, 5: 10}[p]
    mesh = synth.hex_lattice(n, 0.1, seed=110 + p, rotate_seed=210 + p)
    E = mesh["hex"].shape[0]
    kappa = synth.lognormal_iid(E, p + 2, 1.0, seed=111 + p)
    S, X, kc = _setup(mesh, p, kappa)
    div = P.Operator(S, P.DIVERGENCE, S.qdata(P.DIVERGENCE, coeff=kc), constrained=False)
    mass = P.Operator(S, P.MASS, S.qdata(P.MASS, coeff=kc), constrained=False)
    A = np.array([[0.3, -1.1, 0.4], [0.9, 1.7, -0.2], [0.5, 0.8, -2.3]])
    u = X @ A.T + np.array([0.2, -0.7, 1.3])
    y = div.apply(_cuda(np.ascontiguousarray(u.T).ravel())).cpu().numpy()
    m1 = mass.apply(torch.ones(S.ndofs, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert parity_err(y, np.trace(A) * m1) <= 1e-12
    qd1 = S.qdata(P.DIVERGENCE)
    div1 = P.Operator(S, P.DIVERGENCE, qd1, constrained=False)
    uu = np.stack([synth.hash_normal(X, seed=120 + c) for c in range(3)])
    uu[:, S.boundary_dofs()] = 0.0
    q = synth.hash_normal(X, seed=125)
    dq_ = div1.apply(_cuda(uu.ravel())).cpu().numpy()
    # the gradient operator on the same quadrature data
    grad1 = P.Operator(S, P.GRADIENT, qd1, constrained=False)
    gq = grad1.apply(_cuda(q)).cpu().numpy().reshape(3, -1)
    lhs, rhs = float(q @ dq_), -float(np.sum(uu * gq))
    assert abs(lhs - rhs) <= 1e-12 * float(np.abs(q * dq_).sum())
    # and the divergence of a field vanishing on the boundary integrates to zero
    assert abs(float(dq_.sum())) <= 1e-12 * float(np.abs(dq_).sum())


def test_divergence_limits():
    S = P.Space(P.Mesh.from_dict(synth.hex_lattice(2, 0.1, seed=1)), 2)
    qd = S.qdata(P.DIVERGENCE)
    with pytest.raises(P.PafemError):
        P.Operator(S, P.DIVERGENCE, qd)                    # constrained is not defined
    with pytest.raises(P.PafemError):
        P.Operator(S, P.DIVERGENCE, qd, constrained=False, scatter="evec")
    op = P.Operator(S, P.DIVERGENCE, qd, constrained=False)
    with pytest.raises(P.PafemError):
        op.diagonal()
    with pytest.raises(ValueError):
        op.apply(torch.zeros(S.ndofs, dtype=torch.float64, device="cuda"))  # needs 3 * ndofs
    with pytest.raises(P.PafemError):
        P.Operator(S, P.DIVERGENCE, P.lowered_qdata(qd, P.F32), qdata_dtype=P.F32,
                   constrained=False)


def _lame_pairs(E, p, seed):
    lam = synth.lognormal_iid(E, p + 2, 0.5, seed=seed)
    mu = synth.lognormal_iid(E, p + 2, 0.5, seed=seed + 1)
    pairs = np.stack([np.reshape(lam, (E, -1)), np.reshape(mu, (E, -1))], axis=-1)
    return lam, mu, _cuda(pairs.ravel())


@pytest.mark.parametrize("p", range(1, 9))
def test_elasticity_apply(p):
    """Linear elasticity with lognormal lambda and mu per point on rotated jittered
    elements, three-component input: against the oracle's assembled vector operator,
    unconstrained and with every component's essential dofs eliminated, to 1e-12."""
    mesh = synth.hex_lattice(SHAPES[p], 0.1, seed=130 + p, rotate_seed=230 + p)
    E = mesh["hex"].shape[0]
    lam, mu, lm = _lame_pairs(E, p, 131 + p)
    S, X, _ = _setup(mesh, p, renumber=(p % 2 == 1))
    qd = S.qdata(P.ELASTICITY, coeff=lm)
    ref = oracle.H1Space(mesh, p)
    Ke = forms.element_elasticity(mesh, p, p + 2, lam, mu)
    nd = Ke.shape[2]
    V = forms.vector_space(ref)
    K = oracle.assemble(V, Ke.reshape(E, 3 * nd, 3 * nd))
    Xo = ref.dof_coordinates()
    perm = match_by_coords(X, Xo)
    x3 = _cuda(np.concatenate([synth.hash_normal(X, seed=140 + c) for c in range(3)]))
    xo = np.concatenate([synth.hash_normal(Xo, seed=140 + c) for c in range(3)])
    for constrained in (False, True):
        op = P.Operator(S, P.ELASTICITY, qd, constrained=constrained)
        y = op.apply(x3).cpu().numpy().reshape(3, -1)
        A = oracle.constrain(K, np.zeros(V.ndofs), V.boundary)[0] if constrained else K
        want = (A @ xo).reshape(3, -1)[:, perm]
        err = parity_err(y.ravel(), want.ravel())
        print(f"elasticity p={p} constrained={constrained}: rel err {err:.2e}")
        assert err <= TOL


@pytest.mark.parametrize("p", [2, 3, 6])
def test_elasticity_properties_many_tiles(p):
    """At ~1e5 dofs: the six rigid-body fields give K u = 0 (unconstrained, point-varying
    lambda and mu), and the operator is symmetric, <v, K u> = <u, K v>."""
    n = {2: 24, 3: 16, 6: 8}[p]
    mesh = synth.hex_lattice(n, 0.1, seed=150 + p, rotate_seed=250 + p)
    E = mesh["hex"].shape[0]
    _, _, lm = _lame_pairs(E, p, 151 + p)
    S, X, _ = _setup(mesh, p)
    op = P.Operator(S, P.ELASTICITY, S.qdata(P.ELASTICITY, coeff=lm), constrained=False)
    u = _cuda(np.concatenate([synth.hash_normal(X, seed=160 + c) for c in range(3)]))
    Ku = op.apply(u)
    scale = float(Ku.abs().max())
    modes = [np.tile(e_, (S.ndofs, 1)) for e_ in np.eye(3)]
    modes += [np.cross(w, X) for w in np.eye(3)]
    for m in modes:
        r = op.apply(_cuda(m.T.ravel()))
        assert float(r.abs().max()) <= 1e-12 * scale * max(1.0, float(np.abs(m).max()))
    v = _cuda(np.concatenate([synth.hash_normal(X, seed=170 + c) for c in range(3)]))
    a, b = float(v @ Ku), float(u @ op.apply(v))
    assert abs(a - b) <= 1e-12 * float((v.abs() @ Ku.abs()))


def test_elasticity_limits():
    S = P.Space(P.Mesh.from_dict(synth.hex_lattice(2, 0.1, seed=1)), 2)
    E = S.nelem
    _, _, lm = _lame_pairs(E, 2, 5)
    qd = S.qdata(P.ELASTICITY, coeff=lm)
    with pytest.raises(ValueError):
        S.qdata(P.ELASTICITY)                               # needs (lambda, mu)
    with pytest.raises(P.PafemError):
        P.Operator(S, P.ELASTICITY, qd, scatter="evec")
    with pytest.raises(P.PafemError):
        P.Operator(S, P.ELASTICITY, qd, vector=True)        # vector-valued by itself
    op = P.Operator(S, P.ELASTICITY, qd)
    with pytest.raises(P.PafemError):
        op.diagonal()
    with pytest.raises(ValueError):
        op.apply(torch.zeros(S.ndofs, dtype=torch.float64, device="cuda"))  # needs 3 * ndofs
    n3 = 3 * S.ndofs
    with pytest.raises(P.PafemError):
        op.pcg(torch.ones(S.ndofs, dtype=torch.float64, device="cuda"),
               diag=torch.ones(S.ndofs, dtype=torch.float64, device="cuda"))
    y = op.apply(torch.zeros(n3, dtype=torch.float64, device="cuda"))
    assert float(y.abs().max()) == 0.0


def test_degenerate_solves():
    """One p = 1 element (every dof essential): the constrained operator is the identity,
    its diagonal is 1 and CG returns b after one iteration.  A zero right-hand side from a
    zero start is solved with no iteration; from a random start the stop is relative to the
    initial residual and the iterate goes to zero."""
    S1 = P.Space(P.Mesh.from_dict(synth.hex_lattice(1, 0.0)), 1)
    op1 = P.Operator(S1, P.DIFFUSION, S1.qdata(P.DIFFUSION))
    v = _cuda(np.arange(S1.ndofs, dtype=np.float64) + 1.0)
    assert torch.equal(op1.apply(v), v)
    assert torch.equal(op1.diagonal(), torch.ones_like(v))
    x, info = op1.pcg(v, rel_tol=1e-12)
    assert info["status"] == "OK" and info["iters"] <= 1
    assert float((x - v).abs().max()) <= 1e-15 * float(v.abs().max())

    S = P.Space(P.Mesh.from_dict(synth.hex_lattice(4, 0.1, seed=9)), 2)
    op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION))
    zero = torch.zeros(S.ndofs, dtype=torch.float64, device="cuda")
    x, info = op.pcg(zero, rel_tol=1e-10)
    assert info["status"] == "OK" and info["iters"] == 0 and float(x.abs().max()) == 0.0
    x0 = _cuda(synth.hash_normal(S.dof_coords(), seed=3))
    x, info = op.pcg(zero, x=x0.clone(), rel_tol=1e-10, max_iter=5000)
    print(f"zero rhs from a random start: {info['iters']} its, rel res {info['rel_res']:.1e}, "
          f"|x|/|x0| {float(x.norm() / x0.norm()):.1e}")
    assert info["status"] == "OK" and info["iters"] > 0 and info["rel_res"] <= 1e-10
    assert float(x.norm()) <= 1e-6 * float(x0.norm())
