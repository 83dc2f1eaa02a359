"""Element network, learned preconditioner and flexible CG (oracle; test infrastructure only).

None of this is in the paper: the learned preconditioner is an addition to the
paper's CG on partially assembled operators ("Scalable Linear Solvers" notes
that matrix-free operators need matrix-free preconditioners).  Definitions:

* Network N: x -> W3 relu(W2 relu(W1 x + b1) + b2) + b3.
* Element input: x_E = [f_E, 0...], f_E the log-ratios of the coefficient mean over
  the 8 octants of the element's quadrature points to the element mean kbar_E.
* Element weights: c_E = softplus(N(x_E)) (K values, positive).
* Preconditioner, with a learned basis V (one (p+1)^3 x K matrix shared by all
  elements), the element restriction R_E (essential dofs read as 0) and dbar_E the
  mean of diag over the element's non-essential nodes (1 if it has none):
      z = r / diag + sum_E R_E^t V diag(c_E / dbar_E) V^t R_E r,   z = 0 on essential dofs.
  It is linear in r, symmetric, and the correction is positive semidefinite, so
  z(r) is an SPD preconditioner for any network and basis; dividing by dbar_E
  makes it invariant to the scale of the coefficient and to the element size.
* Training loss on a pair (r, e) with A e = r: L = ||A (e - z(r))||^2_{D^-1} /
  ||r||^2_{D^-1} (the error of the correction measured in the norm a local
  preconditioner controls).
* Adam with bias correction.
* Flexible CG with the Polak-Ribiere beta, beta = r_new . (z_new - z_old) / (r . z).

Pins (tests/test_oracle_mlp.py): network backward and the loss gradient (network
and basis) against central finite differences, Adam against its closed form on a
quadratic, V = 0 reproduces Jacobi, the preconditioner is symmetric with a positive
semidefinite correction (brute force on a small mesh), and FCG with a linear SPD
preconditioner matches PCG.
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


def softplus(a):
    return np.logaddexp(0.0, a)


def sigmoid(a):
    return 0.5 * (1.0 + np.tanh(0.5 * a))


def network_inputs(feats, in_dim):
    """X [E, in_dim] = [f_E, 0...]."""
    X = np.zeros((feats.shape[0], in_dim))
    X[:, :feats.shape[1]] = feats
    return X


def diag_mean(diag, elem_dofs, boundary):
    """dbar_E: mean of diag over the element's non-essential nodes (1 if none)."""
    inner = ~boundary[elem_dofs]
    cnt = inner.sum(axis=1)
    tot = (diag[elem_dofs] * inner).sum(axis=1)
    return np.where(cnt > 0, tot / np.maximum(cnt, 1), 1.0)


def precondition(P, V, r, diag, elem_dofs, boundary, feats, in_dim):
    """z = M(r) and the intermediates the gradient needs."""
    X = network_inputs(feats, in_dim)
    a, cache = forward(P, X)
    c = softplus(a)
    dbar = diag_mean(diag, elem_dofs, boundary)
    rz = np.where(boundary, 0.0, r)
    rE = rz[elem_dofs]                       # [E, nd]
    t = rE @ V                               # [E, K]
    w = c / dbar[:, None]
    yE = (w * t) @ V.T                       # [E, nd]
    z = r / diag + np.bincount(elem_dofs.ravel(), weights=yE.ravel(), minlength=r.size)
    z[boundary] = 0.0
    return z, (a, cache, c, dbar, rE, t, w)


def loss_and_grads(P, V, A, r, e, diag, elem_dofs, boundary, feats, in_dim):
    """Training loss L = ||A(e - z)||^2_{D^-1} / ||r||^2_{D^-1}; gradients of the network
    parameters and of the basis V."""
    z, (a, cache, c, dbar, rE, t, w) = precondition(P, V, r, diag, elem_dofs, boundary, feats,
                                                    in_dim)
    u = A @ (e - z)
    rn = r @ (r / diag)
    L = (u @ (u / diag)) / rn
    g = -2.0 * (A @ (u / diag)) / rn          # dL/dz
    g[boundary] = 0.0                         # z is pinned to 0 there
    gE = g[elem_dofs]                         # dL/dy_E
    s = gE @ V                                # V^t g_E
    dV = gE.T @ (w * t) + rE.T @ (w * s)
    dc = s * t / dbar[:, None]
    G = backward(P, cache, dc * sigmoid(a))
    G["V"] = dV
    return L, G


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
