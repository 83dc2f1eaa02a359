"""Pins for the oracle's CG (CPU only): agreement with a sparse direct solve,
monotone A-norm error, and the small Poisson configuration converging."""
import numpy as np
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import forms
from oracle.forms import assemble_vector


def _poisson(n=8, p=2, jitter=0.1, seed=1):
    mesh = synth.hex_lattice(n, jitter, seed=seed)
    s = oracle.H1Space(mesh, p)
    K = oracle.assemble(s, forms.element_stiffness(mesh, p, p + 2))
    b = assemble_vector(s, forms.element_load(mesh, p, p + 2, synth.sine_source))
    Kc, bc = oracle.constrain(K, b, s.boundary)
    return s, Kc, bc


def test_pcg_matches_direct_solve():
    s, A, b = _poisson(n=6, p=2)
    xd = spla.spsolve(A.tocsc(), b)
    res = oracle.pcg(A, b, A.diagonal(), tol=1e-13, maxiter=2000)
    assert res["converged"] and res["true_rel_res"] < 1e-12
    assert np.linalg.norm(res["x"] - xd) / np.linalg.norm(xd) < 1e-11


def test_pcg_error_monotone_in_energy_norm():
    s, A, b = _poisson(n=4, p=3)
    xd = spla.spsolve(A.tocsc(), b)
    errs = []
    for k in range(1, 30):
        r = oracle.pcg(A, b, A.diagonal(), tol=0.0, maxiter=k)
        e = r["x"] - xd
        errs.append(e @ (A @ e))
    assert np.all(np.diff(errs) <= 1e-14 * errs[0])


def test_small_poisson_configuration_converges():
    # unit cube 8^3, 10% jitter, p = 2 (4913 dofs), Jacobi-PCG to 1e-10
    s, A, b = _poisson(n=8, p=2, jitter=0.1, seed=1)
    assert s.ndofs == 4913 and s.boundary.sum() == 1538
    res = oracle.pcg(A, b, A.diagonal(), tol=1e-10, maxiter=2000)
    assert res["converged"] and res["true_rel_res"] < 1e-9
    assert res["history"][-1] <= 1e-10
    err = oracle.l2_error(s, res["x"], synth.sine_solution)
    assert err < 1e-3


def test_host_csr_timing_variant_matches_scipy_and_python_pcg():
    """The C/OpenMP timing variant (oracle/csr_host.c) against scipy's product and the
    Python PCG on a constrained p = 2 diffusion problem."""
    from oracle import csr_host
    csr_host.build_library()
    mesh = synth.hex_lattice(4, 0.1, seed=1)
    sp = oracle.H1Space(mesh, 2)
    K = oracle.assemble(sp, forms.element_stiffness(mesh, 2, 4))
    bv = assemble_vector(sp, forms.element_load(mesh, 2, 4, synth.sine_source))
    Kc, bc = oracle.constrain(K, bv, sp.boundary)
    H = csr_host.HostCSR(Kc)
    x = np.random.default_rng(0).normal(size=sp.ndofs)
    assert np.abs(H.matvec(x) - Kc @ x).max() < 1e-13 * np.abs(Kc @ x).max()
    xs, its, rel = H.pcg_jacobi(bc, Kc.diagonal(), tol=1e-10)
    ref = oracle.pcg(Kc, bc, Kc.diagonal(), tol=1e-10)
    assert rel <= 1e-10 and abs(its - ref["iters"]) <= 1
    assert np.linalg.norm(xs - ref["x"]) <= 1e-8 * np.linalg.norm(ref["x"])
