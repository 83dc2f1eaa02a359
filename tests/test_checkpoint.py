"""Host checkpoints (no GPU): the .npz solve and training records round-trip exactly,
are read without unpickling, refuse a file of the other kind, and an interrupted
write leaves the previous checkpoint in place.  learned.train()'s resume logic
(replayed sample draws and learning-rate decays) is checked with the library calls
replaced by recorders, so that a run split at any step draws the same samples at
the same rates as one that never stopped."""
import json

import numpy as np
import pytest

from paper_1911_09220_amd import checkpoint as ck


def _state(n, seed):
    rng = np.random.default_rng(seed)
    return {"params": rng.normal(size=n).astype(np.float32),
            "adam_m": rng.normal(size=n).astype(np.float32),
            "adam_v": rng.random(n).astype(np.float32), "adam_step": 123}


def test_solve_record_round_trips(tmp_path):
    x = np.random.default_rng(0).normal(size=1000)
    hist = np.geomspace(1.0, 1e-9, 37)
    cfg = {"order": 3, "mesh": "hex_lattice", "jitter": 0.05}
    path = tmp_path / "solve.npz"
    ck.save_solve(path, x, hist, config=cfg, seeds={"mesh": 2, "rhs": 7})
    got = ck.load_solve(path)
    assert got["x"].dtype == np.float64 and np.array_equal(got["x"], x)
    assert np.array_equal(got["history"], hist)
    assert got["config"] == cfg and got["seeds"] == {"mesh": 2, "rhs": 7}
    with np.load(path, allow_pickle=False) as z:  # plain arrays only
        assert all(z[k].dtype != object for k in z.files)


def test_training_record_round_trips_bitwise(tmp_path):
    st = _state(4097, 1)
    path = tmp_path / "train.npz"
    ck.save_training(path, st, train_step=40, seed=33, config={"hidden": 32})
    got = ck.load_training(path)
    for k in ("params", "adam_m", "adam_v"):
        assert got["state"][k].dtype == np.float32
        assert got["state"][k].tobytes() == st[k].tobytes()
    assert got["state"]["adam_step"] == 123
    assert (got["train_step"], got["seed"], got["config"]) == (40, 33, {"hidden": 32})


def test_wrong_kind_and_bad_state_are_refused(tmp_path):
    ck.save_solve(tmp_path / "s.npz", np.zeros(3))
    with pytest.raises(ValueError, match="format"):
        ck.load_training(tmp_path / "s.npz")
    np.savez(tmp_path / "plain.npz", x=np.zeros(3))
    with pytest.raises(ValueError, match="format"):
        ck.load_solve(tmp_path / "plain.npz")
    st = _state(10, 2)
    st["adam_v"] = st["adam_v"][:9]
    with pytest.raises(ValueError, match="length"):
        ck.save_training(tmp_path / "t.npz", st, 1, 0)


def test_interrupted_save_keeps_the_previous_checkpoint(tmp_path, monkeypatch):
    path = tmp_path / "train.npz"
    ck.save_training(path, _state(64, 3), train_step=10, seed=5)

    def broken(f, **arrays):
        f.write(b"partial")
        raise OSError("disk full")

    monkeypatch.setattr(np, "savez", broken)
    with pytest.raises(OSError):
        ck.save_training(path, _state(64, 4), train_step=20, seed=5)
    monkeypatch.undo()
    got = ck.load_training(path)
    assert got["train_step"] == 10
    assert got["state"]["params"].tobytes() == _state(64, 3)["params"].tobytes()


class _Recorder:
    """Stands in for the network and the library calls train() makes."""

    def __init__(self):
        self.calls, self.lrs, self.steps = [], [], 0

    def get_state(self):
        n = 4
        return {"params": np.full(n, self.steps, np.float32), "adam_m": np.zeros(n, np.float32),
                "adam_v": np.zeros(n, np.float32), "adam_step": self.steps}

    def adam_step(self, lr):
        self.lrs.append(lr)
        self.steps += 1


def _run(monkeypatch, tmp_path, start, steps, every=0):
    torch = pytest.importorskip("torch")
    from paper_1911_09220_amd import learned as L
    rec = _Recorder()

    def loss_grad(net, op, feats, diag, r, e, loss, work):
        rec.calls.append(int(r[0]))
        loss.fill_(float(r[0]))

    monkeypatch.setattr(L.P, "_learned_work", lambda op: None)
    monkeypatch.setattr(L.P, "learned_loss_grad", loss_grad)
    samples = [(object(), None, None, torch.full((1,), float(i), dtype=torch.float64), None)
               for i in range(11)]
    path = tmp_path / f"ck_{start}_{steps}.npz"
    losses = L.train(rec, samples, steps=steps, lr=1e-2, lr_decay=0.5, decay_every=7, seed=9,
                     start=start, checkpoint=path, checkpoint_every=every)
    return rec, losses, path


def test_resumed_training_draws_like_an_unbroken_run(monkeypatch, tmp_path):
    full, lf, _ = _run(monkeypatch, tmp_path, 0, 30)
    assert len(full.calls) == 30 and len(set(full.calls)) > 5
    assert full.lrs[0] == 1e-2 and full.lrs[7] == 5e-3 and full.lrs[29] == 1e-2 / 16
    for cut in (1, 7, 13, 29):
        a, la, pa = _run(monkeypatch, tmp_path, 0, cut)
        b, lb, _ = _run(monkeypatch, tmp_path, cut, 30 - cut)
        assert a.calls + b.calls == full.calls
        assert a.lrs + b.lrs == full.lrs
        assert np.array_equal(np.concatenate([la, lb]), lf)
        assert ck.load_training(pa)["train_step"] == cut


def test_periodic_checkpoints_mark_the_step_reached(monkeypatch, tmp_path):
    saved = []
    real = ck.save_training

    def spy(path, state, train_step, seed, config=None):
        saved.append((train_step, state["adam_step"], seed))
        real(path, state, train_step, seed, config)

    monkeypatch.setattr(ck, "save_training", spy)
    _run(monkeypatch, tmp_path, 5, 20, every=6)
    assert saved == [(6, 1, 9), (12, 7, 9), (18, 13, 9), (24, 19, 9), (25, 20, 9)]
    assert json.loads(json.dumps(saved))  # plain integers
