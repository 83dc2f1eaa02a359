"""Jacobi-PCG status codes and run-to-run reproducibility on the GPU.

* ENOTCONV: the iteration limit reached before the tolerance, with the result filled in.
* EBREAKDOWN: the operator of negated quadrature data is negative definite on the free
  dofs, so the first step's p . A p is negative ("Scalable Linear Solvers": CG needs an
  SPD operator) and the solve stops at once.
* The deterministic scatter (element vectors gathered per dof in a fixed order) and the
  solver's fixed-order grid reductions make the whole solve bitwise reproducible.  The
  default atomic scatter sums each dof's element contributions in arrival order, so two
  solves differ at rounding level; their solutions are bound to agree far inside the
  distance 2 kappa(A) rel_tol that the stopping test alone would allow.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import pafem as P  # noqa: E402


def _problem(scatter="atomic", negate=False):
    mesh = synth.hex_lattice(8, 0.1, seed=1)
    S = P.Space(P.Mesh.from_dict(mesh), 2)
    qd = S.qdata(P.DIFFUSION)
    if negate:
        qd = -qd
    op = P.Operator(S, P.DIFFUSION, qd, scatter=scatter)
    return S, op, S.linear_form(P.SOURCE_SINE)


def test_pcg_iteration_limit_reports_enotconv():
    S, op, b = _problem()
    x, info = op.pcg(b, rel_tol=1e-10, max_iter=1)
    print(info["status"], info["iters"], info["rel_res"])
    assert info["status"] == "ENOTCONV" and not info["converged"]
    assert info["iters"] == 1 and np.isfinite(info["rel_res"]) and info["rel_res"] > 1e-10
    assert bool(torch.isfinite(x).all()) and float(x.abs().max()) > 0.0
    # the result is filled in: the reported residual is that of the returned iterate
    # (CG lowers the error's energy norm; the residual's 2-norm may grow in one step)
    true = float((b - op.apply(x)).norm() / b.norm())
    assert abs(true - info["rel_res"]) <= 1e-10 * true


@pytest.mark.parametrize("precond", [P.PRECOND_JACOBI, P.PRECOND_NONE])
def test_pcg_on_negative_definite_operator_reports_ebreakdown(precond):
    S, op, b = _problem(negate=True)
    x, info = op.pcg(b, rel_tol=1e-10, max_iter=100, precond=precond)
    print(info["status"], info["iters"])
    assert info["status"] == "EBREAKDOWN" and not info["converged"]
    assert info["iters"] <= 1


def test_deterministic_scatter_solve_is_bitwise_reproducible():
    S, op, b = _problem(scatter="evec")
    x1, i1 = op.pcg(b, rel_tol=1e-10, max_iter=500)
    x2, i2 = op.pcg(b, rel_tol=1e-10, max_iter=500)
    assert i1["status"] == "OK" and i1["iters"] == i2["iters"]
    assert np.array_equal(i1["history"], i2["history"])
    assert torch.equal(x1, x2)


def test_atomic_scatter_solves_agree_to_rounding():
    S, op, b = _problem()
    xs, its = [], []
    for _ in range(3):
        x, info = op.pcg(b, rel_tol=1e-10, max_iter=500)
        assert info["status"] == "OK"
        xs.append(x)
        its.append(info["iters"])
    worst = max(float((xs[k] - xs[0]).norm() / xs[0].norm()) for k in range(1, 3))
    print(f"iterations {its}, largest solution difference {worst:.2e}")
    assert max(its) - min(its) <= 1
    assert worst <= 1e-9
