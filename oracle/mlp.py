"""Element-patch network, learned preconditioner and flexible CG (oracle; test infrastructure only).

None of this is in the paper: the learned preconditioner is an addition to the
paper's CG on partially assembled operators ("Scalable Linear Solvers" notes
that matrix-free operators need matrix-free preconditioners).  Definitions:

* Network N: x -> W3 relu(W2 relu(W1 x + b1) + b2) + b3.
* Element input: x_E = [r_E / s_E, f_E, 0...] with s_E = ||r_E||_2 (+tiny) and f_E
  the log-ratios of the coefficient mean over the 8 octants of the element's
  quadrature points to the element mean kbar_E.
* Preconditioner: z = r / diag + G^t( w * (s_E / kbar_E) * N(x_E) ), w = 1/m_g
  (m_g = number of element nodes sharing dof g); z = 0 on essential dofs.
* Training loss on a pair (r, e) with A e = r: L = ||A (e - z(r))||^2_{D^-1} /
  ||r||^2_{D^-1} (the error of the correction measured in the norm a local
  preconditioner controls).
* Adam with bias correction.
* Flexible CG with the Polak-Ribiere beta, beta = r_new . (z_new - z_old) / (r . z).

Pins (tests/test_oracle_mlp.py): backward against central finite differences,
Adam against its closed form on a quadratic, a zero last layer reproduces Jacobi,
and FCG with a linear SPD preconditioner matches PCG.
"""
import numpy as np


def forward(P, X):
    Z1 = X @ P["W1"].T + P["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ P["W2"].T + P["b2"]
    H2 = np.maximum(Z2, 0.0)
    out = H2 @ P["W3"].T + P["b3"]
    return out, (X, Z1, H1, Z2, H2)


def backward(P, cache, dout):
    X, Z1, H1, Z2, H2 = cache
    g = {"W3": dout.T @ H2, "b3": dout.sum(axis=0)}
    dZ2 = (dout @ P["W3"]) * (Z2 > 0)
    g["W2"] = dZ2.T @ H1
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W2"]) * (Z1 > 0)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam_step(P, G, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place; state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in P:
        m = state.setdefault("m_" + k, np.zeros_like(P[k]))
        v = state.setdefault("v_" + k, np.zeros_like(P[k]))
        m *= beta1
        m += (1 - beta1) * G[k]
        v *= beta2
        v += (1 - beta2) * G[k] ** 2
        mhat = m / (1 - beta1 ** t)
        vhat = v / (1 - beta2 ** t)
        P[k] -= lr * mhat / (np.sqrt(vhat) + eps)
    return P


def element_features(kappa, q1d):
    """kbar [E] and the 8 octant log-ratio features [E, 8] from kappa [E, Q^3]."""
    E = kappa.shape[0]
    k = kappa.reshape(E, q1d, q1d, q1d)          # [e, qz, qy, qx]
    half = q1d // 2
    feats = np.empty((E, 8))
    kbar = kappa.mean(axis=1)
    for o in range(8):
        sx = slice(half, None) if o & 1 else slice(0, half)
        sy = slice(half, None) if o & 2 else slice(0, half)
        sz = slice(half, None) if o & 4 else slice(0, half)
        feats[:, o] = np.log(k[:, sz, sy, sx].reshape(E, -1).mean(axis=1) / kbar)
    return kbar, feats


def patch_inputs(r, elem_dofs, feats, in_dim, tiny=1e-300):
    """Network inputs [E, in_dim] and the element scales s_E."""
    rE = r[elem_dofs]
    s = np.sqrt((rE ** 2).sum(axis=1)) + tiny
    X = np.zeros((rE.shape[0], in_dim))
    nd = rE.shape[1]
    X[:, :nd] = rE / s[:, None]
    X[:, nd:nd + feats.shape[1]] = feats
    return X, s


def multiplicity(elem_dofs, ndofs):
    return np.bincount(elem_dofs.ravel(), minlength=ndofs).astype(np.float64)


def precondition(P, r, diag, elem_dofs, boundary, feats, kbar, in_dim):
    """z = M(r).  Only the first (p+1)^3 network outputs are used (one per element node)."""
    X, s = patch_inputs(r, elem_dofs, feats, in_dim)
    out, cache = forward(P, X)
    nd = elem_dofs.shape[1]
    m = multiplicity(elem_dofs, r.size)
    scale = (s / kbar)[:, None]
    contrib = np.bincount(elem_dofs.ravel(), weights=(scale * out[:, :nd]).ravel(),
                          minlength=r.size)
    z = r / diag + contrib / m
    z[boundary] = 0.0
    return z, (X, s, cache, m, scale)


def loss_and_grads(P, A, r, e, diag, elem_dofs, boundary, feats, kbar, in_dim):
    """Training loss L = ||A(e - z)||^2_{D^-1} / ||r||^2_{D^-1} and its parameter gradients."""
    z, (X, s, cache, m, scale) = precondition(P, r, diag, elem_dofs, boundary, feats, kbar, in_dim)
    u = A @ (e - z)
    rn = r @ (r / diag)
    L = (u @ (u / diag)) / rn
    dz = -2.0 * (A @ (u / diag)) / rn
    dz[boundary] = 0.0
    nd = elem_dofs.shape[1]
    dout = np.zeros((elem_dofs.shape[0], P["W3"].shape[0]))
    dout[:, :nd] = scale * (dz / m)[elem_dofs]
    return L, backward(P, cache, dout)


def fcg(A, b, precond, tol=1e-8, maxiter=2000):
    """Flexible CG, x0 = 0; stop on ||r|| <= tol ||b||.  Returns x, iterations, history."""
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    z = precond(r)
    p = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r) / bn]
    k = 0
    while hist[-1] > tol and k < maxiter:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r_new = r - alpha * q
        z_new = precond(r_new)
        beta = (r_new @ (z_new - z)) / rz
        rz = r_new @ z_new
        p = z_new + beta * p
        r, z = r_new, z_new
        k += 1
        hist.append(np.linalg.norm(r) / bn)
    return x, k, hist
