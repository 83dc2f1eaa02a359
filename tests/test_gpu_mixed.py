"""Reduced-precision inner operators and FP64 iterative refinement on the GPU.

* f64 -> f32 / bf16 conversion is bit-exact against the oracle's rounding;
* the FP32 and BF16-qdata applies are compared with the FP64 oracle and the error
  is stated per result (bounds: FP32 arithmetic 1e-5, BF16 quadrature data 1e-2,
  i.e. a few units of the 2^-8 bf16 roundoff);
* iterative refinement reaches an FP64 residual of 1e-10 and its solution matches
  the oracle's direct solve to kappa * 1e-10.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.precision import to_bf16_bits, to_f32
from tests._common import OracleProblem, match_by_coords, rel_err, parity_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_conversion_bit_exact():
    x = np.random.default_rng(3).lognormal(0.0, 4.0, size=100003) * np.sign(
        np.random.default_rng(4).normal(size=100003))
    x[:4] = [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 0.0, -7.25]
    xd = _cuda(x)
    f = P.lowered_qdata(xd, P.F32).cpu().numpy()
    np.testing.assert_array_equal(f.view(np.uint32), to_f32(x).view(np.uint32))
    b = P.lowered_qdata(xd, P.BF16).cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(b, to_bf16_bits(x))


@pytest.mark.parametrize("p", [1, 3, 6])
@pytest.mark.parametrize("dtype,tol", [(P.F32, 1e-5), (P.BF16, 1e-2)])
def test_reduced_precision_apply(p, dtype, tol):
    shape = {1: (5, 4, 4), 3: (4, 3, 3), 6: (2, 2, 2)}[p]
    mesh = synth.hex_lattice(shape, 0.1, seed=50 + p, rotate_seed=51)
    kappa = synth.lognormal_iid(mesh["hex"].shape[0], p + 2, 1.0, seed=52)
    S = P.Space(P.Mesh.from_dict(mesh), p)
    X = S.dof_coords()
    qd = S.qdata(P.DIFFUSION, coeff=_cuda(kappa))
    lo = P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, dtype), qdata_dtype=dtype)
    x = synth.hash_normal(X, seed=53)
    y = lo.apply(torch.as_tensor(x, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    ref = OracleProblem(mesh, p, coeff=kappa)
    perm = match_by_coords(X, ref.coords)
    err = parity_err(y, (ref.Kc @ synth.hash_normal(ref.coords, seed=53))[perm])
    print(f"p={p} dtype={'f32' if dtype == P.F32 else 'bf16'} apply rel err vs FP64 oracle {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("keep", [True, False], ids=["reliable", "restart"])
@pytest.mark.parametrize("dtype", [P.F32, P.BF16])
@pytest.mark.parametrize("case", ["poisson", "q2"])
def test_iterative_refinement(case, dtype, keep):
    if case == "poisson":
        mesh, p = synth.hex_lattice(8, 0.1, seed=1), 2
    else:
        mesh, p = synth.q2_warped_lattice(3, 0.05), 6
    S = P.Space(P.Mesh.from_dict(mesh), p)
    X = S.dof_coords()
    qd = S.qdata(P.DIFFUSION)
    hi = P.Operator(S, P.DIFFUSION, qd)
    lo = P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, dtype), qdata_dtype=dtype)
    b = S.linear_form(P.SOURCE_SINE)
    x, info = hi.ir_solve(lo, b, rel_tol=1e-10, inner_rel_tol=1e-2, keep_direction=keep)
    assert info["status"] == "OK" and info["converged"] and info["rel_res"] <= 1e-10
    # the residual history is monotone and the reported residual is the FP64 one
    h = info["history"]
    assert np.all(np.diff(h) < 0)
    r = b - hi.apply(x)
    assert abs(float(r.norm() / b.norm()) - info["rel_res"]) <= 1e-3 * info["rel_res"]
    ref = OracleProblem(mesh, p)
    perm = match_by_coords(X, ref.coords)
    xd = spla.spsolve(ref.Kc.tocsc(), ref.load(synth.sine_source))
    err = rel_err(x.cpu().numpy(), xd[perm])
    print(f"{case} {'f32' if dtype == P.F32 else 'bf16'} keep={keep}: {info['outer']} steps, "
          f"{info['inner_total']} inner its, solution rel err vs oracle {err:.2e}")
    assert err <= 1e-8


def test_refinement_reports_nonconvergence():
    mesh = synth.hex_lattice(4, 0.1, seed=1)
    S = P.Space(P.Mesh.from_dict(mesh), 2)
    qd = S.qdata(P.DIFFUSION)
    hi = P.Operator(S, P.DIFFUSION, qd)
    lo = P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, P.BF16), qdata_dtype=P.BF16)
    b = S.linear_form(P.SOURCE_SINE)
    x, info = hi.ir_solve(lo, b, rel_tol=1e-14, max_outer=1)
    assert info["status"] == "ENOTCONV" and info["outer"] == 1 and not info["converged"]
    assert info["rel_res"] < 1e-1


@pytest.mark.parametrize("dtype", [P.F32, P.BF16])
def test_reliable_update_keeps_pcg_iteration_count(dtype):
    """With an FP32 apply, keeping the inner direction across residual replacements
    keeps the total inner iteration count near FP64 Jacobi-PCG's (a restart every
    step loses the Krylov space and needs more).  With a BF16 operator (apply error
    ~4e-3) both strategies must converge to the same solution; their counts are
    reported."""
    mesh, p = synth.hex_lattice(12, 0.1, seed=3), 3
    S = P.Space(P.Mesh.from_dict(mesh), p)
    kappa = torch.as_tensor(synth.lognormal_iid(S.nelem, p + 2, 1.0, seed=4), device="cuda")
    qd = S.qdata(P.DIFFUSION, coeff=kappa)
    hi = P.Operator(S, P.DIFFUSION, qd)
    lo = P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, dtype), qdata_dtype=dtype)
    b = S.linear_form(P.SOURCE_SINE)
    diag = hi.diagonal()
    x64, i64 = hi.pcg(b, diag=diag, rel_tol=1e-8)
    xk, keep = hi.ir_solve(lo, b, diag=diag, rel_tol=1e-8, keep_direction=True)
    xr, rest = hi.ir_solve(lo, b, diag=diag, rel_tol=1e-8, keep_direction=False)
    print(f"FP64 PCG {i64['iters']} its; reliable {keep['inner_total']} inner / {keep['outer']} "
          f"steps; restart {rest['inner_total']} inner / {rest['outer']} steps")
    assert keep["converged"] and rest["converged"]
    if dtype == P.F32:
        assert keep["inner_total"] <= 1.15 * i64["iters"] + 10
        assert keep["inner_total"] < rest["inner_total"]
    assert float((xk - xr).norm() / xr.norm()) < 1e-6
    assert float((xk - x64).norm() / x64.norm()) < 1e-6
