"""Training orchestration for the learned element preconditioner.

Only sequencing and the initial parameters live here; every computation is a
library call:
* pairs (r_k, e_k = x* - x_k) come from plain Jacobi-PCG runs (pafem_pcg_solve)
  stopped after k iterations, x* from a run to a tight tolerance;
* each training step is pafem_learned_loss_grad (preconditioner forward, the
  A-weighted error loss, backward through the operator and the network) followed
  by pafem_net_adam_step.
"""
from __future__ import annotations

import numpy as np

from . import pafem as P


def initial_params(net, seed=0, bias=-3.0):
    """Starting point: He-normal hidden layers, a zero last layer whose bias makes
    every element weight softplus(bias) (small: the preconditioner starts close to
    Jacobi), and a random basis with unit expected column norm."""
    rng = np.random.default_rng(seed)
    h, i, o = net.hidden, net.in_dim, net.out_dim
    nd = (net.order + 1) ** 3
    return {"W1": rng.normal(scale=np.sqrt(2.0 / i), size=(h, i)), "b1": np.zeros(h),
            "W2": rng.normal(scale=np.sqrt(2.0 / h), size=(h, h)), "b2": np.zeros(h),
            "W3": np.zeros((o, h)), "b3": np.full(o, bias),
            "V": rng.normal(scale=1.0 / np.sqrt(nd), size=(nd, o))}


def jacobi_pairs(op, b, diag, stops=(2, 5, 10, 20, 40, 80), tight=1e-12, max_iter=20000):
    """[(r_k, e_k)] for the listed iteration counts of Jacobi-PCG from x0 = 0."""
    xstar, info = op.pcg(b, diag=diag, rel_tol=tight, max_iter=max_iter, history=False)
    pairs = []
    for k in stops:
        if k >= info["iters"]:
            break
        xk, _ = op.pcg(b, diag=diag, rel_tol=0.0, max_iter=k, history=False)
        ek = xstar - xk
        rk = op.apply(ek)
        pairs.append((rk, ek))
    return pairs


class CompactFields:
    """Training data of many coefficient fields kept small: per field the coefficient,
    the element features, the diagonal and its pairs in FP32; one quadrature-data buffer
    and one operator are shared, and the buffer is re-assembled from the drawn field's
    coefficient (a few ms) when a sample of another field is drawn.  For field counts
    whose operators would not all fit in device memory (1.6 GB each at 64^3, p = 3)."""

    def __init__(self, space, kind=P.DIFFUSION):
        self.space, self.kind = space, kind
        self.qd = space.qdata(kind)
        self.op = P.Operator(space, kind, self.qd)
        self.fields, self.samples, self.current = [], [], None

    def use(self, f):
        """The shared operator, its quadrature data set to field f."""
        if self.current != f:
            P.pafem_qdata_assemble(self.space.handle, self.kind, self.space.p + 2,
                                   self.fields[f][0], 1.0, self.qd)
            self.current = f
        return self.op

    def add_field(self, kappa, feats, make_pairs):
        """Register a field; make_pairs(op, diag) yields its (r, e) pairs, computed
        with the shared operator set to this field."""
        self.fields.append((kappa, feats, None))
        f = len(self.fields) - 1
        op = self.use(f)
        diag = op.diagonal()
        self.fields[f] = (kappa, feats, diag)
        for r, e in make_pairs(op, diag):
            self.samples.append((f, r.float(), e.float()))

    def __len__(self):
        return len(self.samples)

    def draw(self, i):
        f, r, e = self.samples[i]
        kappa, feats, diag = self.fields[f]
        return self.use(f), feats, diag, r.double(), e.double()

    def without_features(self, zero):
        """The same samples drawn with the element features replaced by `zero` (one
        zeroed feature array): the network's output is then one weight vector for every
        element, the ablation of the network."""
        return _ZeroFeatures(self, zero)


class _ZeroFeatures:
    def __init__(self, store, zero):
        self.store, self.zero, self.qd = store, zero, store.qd

    def __len__(self):
        return len(self.store)

    def draw(self, i):
        op, _, diag, r, e = self.store.draw(i)
        return op, self.zero, diag, r, e


def train(net, samples, steps=500, lr=2e-3, lr_decay=0.5, decay_every=200, seed=0, log_every=0,
          log=print, start=0, checkpoint=None, checkpoint_every=0):
    """Adam on the loss of randomly drawn samples.

    samples: list of (op, feats, diag, r, e), a CompactFields or its without_features()
    view.  start: the training step to begin at; the sample draws and learning-rate
    decays of the steps before it are replayed without work, so a run resumed at a
    checkpoint's train_step (network state restored with Net.set_state) draws the
    same samples at the same rates as one that never stopped.  checkpoint: a path that
    receives the training state (checkpoint.save_training) every checkpoint_every
    steps and at the end.  Returns the losses of steps start .. start + steps - 1
    (host).
    """
    import torch
    from . import checkpoint as ckpt
    rng = np.random.default_rng(seed)
    works = {}
    compact = isinstance(samples, (CompactFields, _ZeroFeatures))
    device = samples.qd.device if compact else samples[0][3].device
    loss_dev = torch.zeros(steps, dtype=torch.float64, device=device)
    cur_lr = lr
    for t in range(start + steps):
        if decay_every and t and t % decay_every == 0:
            cur_lr *= lr_decay
        i = int(rng.integers(len(samples)))
        if t < start:
            continue
        op, feats, diag, r, e = samples.draw(i) if compact else samples[i]
        w = works.get(id(op))
        if w is None:
            w = works[id(op)] = P._learned_work(op)
        P.learned_loss_grad(net, op, feats, diag, r, e, loss=loss_dev[t - start:t - start + 1],
                            work=w)
        net.adam_step(cur_lr)
        if log_every and (t + 1) % log_every == 0:
            log(f"train step {t + 1}: loss {float(loss_dev[t - start]):.4f}")
        if checkpoint is not None and (t + 1 == start + steps or
                                       (checkpoint_every and (t + 1) % checkpoint_every == 0)):
            ckpt.save_training(checkpoint, net.get_state(), t + 1, seed)
    return loss_dev.cpu().numpy()
