"""Checkpoints kept on the host as .npz files of plain arrays (no pickled objects; read
back with numpy's allow_pickle=False):

* a solve: its configuration (JSON text), the seeds, the solution and the residual
  history, so a later PCG can warm-start from the saved solution;
* training of the learned preconditioner: the network's parameters, Adam's moment
  estimates and step count, the training step reached and the sampling seed, so
  learned.train() resumes where it stopped.

Files are written to a temporary name beside the target and renamed into place, so
an interrupted save leaves the previous checkpoint whole.
"""
from __future__ import annotations

import json
import os

import numpy as np

SOLVE_FORMAT = "pafem-solve-1"
TRAIN_FORMAT = "pafem-train-1"


def _host(a, dtype):
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _write(path, arrays):
    path = os.fspath(path)
    tmp = path + ".part"
    with open(tmp, "wb") as f:
        np.savez(f, **arrays)
    os.replace(tmp, path)


def _read(path, fmt):
    with np.load(os.fspath(path), allow_pickle=False) as z:
        got = str(z["format"]) if "format" in z.files else None
        if got != fmt:
            raise ValueError(f"{path}: format {got!r}, expected {fmt!r}")
        return {k: z[k] for k in z.files}


def save_solve(path, x, history=None, config=None, seeds=None):
    """x: the solution (device tensor or array, stored FP64); history: residual norms
    per iteration; config, seeds: JSON-serialisable dicts."""
    _write(path, {"format": np.array(SOLVE_FORMAT),
                  "x": _host(x, np.float64),
                  "history": _host([] if history is None else history, np.float64),
                  "config": np.array(json.dumps(config or {}, sort_keys=True)),
                  "seeds": np.array(json.dumps(seeds or {}, sort_keys=True))})


def load_solve(path):
    """{"x", "history", "config", "seeds"} as saved."""
    z = _read(path, SOLVE_FORMAT)
    return {"x": z["x"], "history": z["history"], "config": json.loads(str(z["config"])),
            "seeds": json.loads(str(z["seeds"]))}


def save_training(path, state, train_step, seed, config=None):
    """state: Net.get_state(); train_step: steps of learned.train() taken so far;
    seed: the sampling seed train() was given."""
    if not (len(state["params"]) == len(state["adam_m"]) == len(state["adam_v"])):
        raise ValueError("parameter and moment arrays differ in length")
    _write(path, {"format": np.array(TRAIN_FORMAT),
                  "params": _host(state["params"], np.float32),
                  "adam_m": _host(state["adam_m"], np.float32),
                  "adam_v": _host(state["adam_v"], np.float32),
                  "adam_step": np.array(int(state["adam_step"]), dtype=np.int64),
                  "train_step": np.array(int(train_step), dtype=np.int64),
                  "seed": np.array(int(seed), dtype=np.int64),
                  "config": np.array(json.dumps(config or {}, sort_keys=True))})


def load_training(path):
    """{"state" (for Net.set_state), "train_step", "seed", "config"} as saved."""
    z = _read(path, TRAIN_FORMAT)
    state = {"params": z["params"], "adam_m": z["adam_m"], "adam_v": z["adam_v"],
             "adam_step": int(z["adam_step"])}
    return {"state": state, "train_step": int(z["train_step"]), "seed": int(z["seed"]),
            "config": json.loads(str(z["config"]))}
