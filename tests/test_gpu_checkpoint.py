"""Checkpoint and resume on the GPU.

* Training of the learned preconditioner stopped at a checkpoint and resumed in a
  fresh network (parameters, Adam moments and step count restored through
  pafem_net_set_state) continues like the run that never stopped: the same losses
  and final parameters up to the order of the atomic sums in the preconditioner
  (bar 1e-6 relative on losses, 1e-5 on parameters, the same bar as the other
  training-equivalence test).  A restart that restores only the parameters (Adam
  state cleared) is shown to miss that bar, so the test sees a lost Adam state.
* The state read back after set_state is bit for bit the state written.
* A PCG solution saved at a loose tolerance and loaded again warm-starts PCG to the
  tight tolerance in fewer iterations than a cold start, to the same solution.
"""
import numpy as np
import pytest

import synth
from tests._common import rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1911_09220_amd import checkpoint as ck  # noqa: E402
from paper_1911_09220_amd import learned as L  # noqa: E402
from paper_1911_09220_amd import pafem as P  # noqa: E402


def _flat(net):
    return np.concatenate([v.ravel() for v in net.get_params().values()])


def test_training_resumes_from_a_checkpoint(tmp_path):
    p, n = 2, 4
    mesh = synth.hex_lattice(n, 0.05, seed=41)
    E = mesh["hex"].shape[0]
    S = P.Space(P.Mesh.from_dict(mesh), p)
    pts = synth.lattice_quadrature_points(n, p + 2)
    b = S.linear_form(P.SOURCE_SINE)
    samples = []
    for f in range(2):
        kappa = synth.grf_lognormal(pts, 0.1, 1e3, seed=1200 + f, device="cuda")
        kappa = kappa.reshape(E, -1).contiguous()
        feats = P.learned_features(S, kappa)
        op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION, coeff=kappa))
        diag = op.diagonal()
        samples += [(op, feats, diag, r, e) for r, e in L.jacobi_pairs(op, b, diag, stops=(2, 5, 10))]
    kw = dict(lr=2e-3, lr_decay=0.5, decay_every=15, seed=43)

    def fresh():
        net = P.Net(p, hidden=32, max_rows=E, max_train_rows=E)
        net.set_params(L.initial_params(net, seed=42))
        return net

    full = fresh()
    loss_full = L.train(full, samples, steps=40, **kw)
    first = fresh()
    path = tmp_path / "train.npz"
    L.train(first, samples, steps=20, checkpoint=path, checkpoint_every=8, **kw)
    saved = ck.load_training(path)
    assert saved["train_step"] == 20 and saved["seed"] == 43
    assert saved["state"]["adam_step"] == 20

    resumed = P.Net(p, hidden=32, max_rows=E, max_train_rows=E)
    resumed.set_state(saved["state"])
    back = resumed.get_state()
    for k in ("params", "adam_m", "adam_v"):
        assert back[k].tobytes() == saved["state"][k].tobytes()
    assert back["adam_step"] == 20
    loss_res = L.train(resumed, samples, steps=20, start=saved["train_step"], **kw)

    cold = P.Net(p, hidden=32, max_rows=E, max_train_rows=E)
    cold.set_params(saved["state"]["params"])
    loss_cold = L.train(cold, samples, steps=20, start=20, **kw)

    d_res = rel_err(_flat(resumed), _flat(full))
    d_cold = rel_err(_flat(cold), _flat(full))
    l_res = float(np.max(np.abs(loss_res - loss_full[20:]) / np.abs(loss_full[20:])))
    l_cold = float(np.max(np.abs(loss_cold - loss_full[20:]) / np.abs(loss_full[20:])))
    print(f"resume: params {d_res:.2e}, losses {l_res:.2e}; "
          f"params-only restart: params {d_cold:.2e}, losses {l_cold:.2e}")
    assert np.all(np.isfinite(loss_full))
    assert l_res <= 1e-6 and d_res <= 1e-5
    assert d_cold > 1e-5


def test_bad_state_is_refused():
    net = P.Net(2, hidden=32, max_rows=8, max_train_rows=8)
    st = net.get_state()
    with pytest.raises(ValueError):
        net.set_state({**st, "adam_v": st["adam_v"][:-1]})
    with pytest.raises(P.PafemError):
        net.set_state({**st, "adam_step": -1})


def test_saved_solution_warm_starts_pcg(tmp_path):
    mesh = synth.hex_lattice(8, 0.1, seed=3)
    S = P.Space(P.Mesh.from_dict(mesh), 3)
    op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION))
    b = S.linear_form(P.SOURCE_SINE)
    diag = op.diagonal()
    x1, i1 = op.pcg(b, diag=diag, rel_tol=1e-5, max_iter=2000)
    assert i1["converged"]
    path = tmp_path / "solve.npz"
    ck.save_solve(path, x1, i1["history"], config={"order": 3, "n": 8, "rel_tol": 1e-5},
                  seeds={"mesh": 3})
    rec = ck.load_solve(path)
    assert rec["config"]["order"] == 3 and len(rec["history"]) == i1["iters"] + 1
    x0 = torch.as_tensor(rec["x"], device="cuda")
    assert torch.equal(x0, x1)
    xw, iw = op.pcg(b, x=x0, diag=diag, rel_tol=1e-10, max_iter=2000)
    xc, ic = op.pcg(b, diag=diag, rel_tol=1e-10, max_iter=2000)
    print(f"warm start: {iw['iters']} its, cold: {ic['iters']} its")
    assert iw["converged"] and ic["converged"]
    assert iw["iters"] < ic["iters"]
    assert float((xw - xc).norm() / xc.norm()) < 1e-8
