"""Plain FP64 oracle of the learned current surrogate (test infrastructure).

THIS MODULE IS TEST INFRASTRUCTURE: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it. It shares no code with the HIP
library.

The surrogate replaces the microscopic cell of the multiscale coupling
(Sec. 5, Eqs. Maxwell_ms and TDKS_ms) by a map from the recent history of the
vector potential at one macroscopic point to the current there. The paper has
no such network; the form taken here is a reading:

* input x = (A(t_{n-W+1}), ..., A(t_n)) / a_scale, a causal window of W
  macroscopic samples (zeros before t = 0);
* a causal convolution with kernel length W evaluated at one output time, i.e.
  a dense layer W -> H, tanh; a dense layer H -> H, tanh; a dense output
  H -> 1; plus a linear skip W -> 1 that carries the linear response;
* y = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3 + ws . x, and I(t_n) = j_scale y;
* loss = mean over the batch of (y - target)^2;
* Adam (Kingma and Ba, ICLR 2015, Algorithm 1) with bias correction.

Flat parameter layout (also the library's): W1 [H][W], b1 [H], W2 [H][H],
b2 [H], w3 [H], b3 [1], ws [W].
"""
from __future__ import annotations

import numpy as np


def n_params(W, H):
    return H * W + H + H * H + H + H + 1 + W


def unpack(theta, W, H):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0

    def take(n, shape):
        nonlocal o
        v = theta[o:o + n].reshape(shape)
        o += n
        return v
    W1 = take(H * W, (H, W))
    b1 = take(H, (H,))
    W2 = take(H * H, (H, H))
    b2 = take(H, (H,))
    w3 = take(H, (H,))
    b3 = take(1, (1,))
    ws = take(W, (W,))
    assert o == theta.shape[0]
    return W1, b1, W2, b2, w3, b3, ws


def pack(W1, b1, W2, b2, w3, b3, ws):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(w3),
                           np.ravel(b3), np.ravel(ws)]).astype(np.float64)


def forward(theta, x, W, H):
    """y for a batch x [B][W]; also returns the hidden activations."""
    W1, b1, W2, b2, w3, b3, ws = unpack(theta, W, H)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.tanh(x @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ w3 + b3[0] + x @ ws
    return y, h1, h2


def loss_and_grad(theta, x, target, W, H):
    """Mean squared error and its gradient by the chain rule, layer by layer."""
    W1, b1, W2, b2, w3, b3, ws = unpack(theta, W, H)
    x = np.asarray(x, dtype=np.float64)
    B = x.shape[0]
    y, h1, h2 = forward(theta, x, W, H)
    r = y - np.asarray(target, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B                       # dL/dy
    g_w3 = h2.T @ dy
    g_b3 = np.array([dy.sum()])
    g_ws = x.T @ dy
    dz2 = np.outer(dy, w3) * (1.0 - h2 * h2)
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    g_W1 = dz1.T @ x
    g_b1 = dz1.sum(axis=0)
    return loss, pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3, g_ws)


def adam_step(theta, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def windows(A, J, W, a_scale=1.0, j_scale=1.0):
    """Training samples from trajectories A, J [n_traj][T]: for every (traj, t)
    the causal window of A ending at t (zeros before 0), and J(t); both scaled.
    Samples are ordered traj-major, then t."""
    A = np.asarray(A, dtype=np.float64)
    J = np.asarray(J, dtype=np.float64)
    n_traj, T = A.shape
    X = np.zeros((n_traj * T, W))
    Y = np.empty(n_traj * T)
    for i in range(n_traj):
        for t in range(T):
            lo = t - W + 1
            seg = A[i, max(lo, 0):t + 1]
            X[i * T + t, W - seg.shape[0]:] = seg / a_scale
            Y[i * T + t] = J[i, t] / j_scale
    return X, Y


def fit_linear(A, J, W, a_scale, j_scale, a_fit, lambda_rel=1e-10):
    """Least-squares linear response for the skip weights and the output bias:
    minimise sum (ws . x + b3 - y)^2 + lambda |(ws, b3)|^2 over every sample
    (causal window x, scaled target y) of the trajectories whose largest |A|
    is within a_fit, lambda = lambda_rel times the mean diagonal of the normal
    matrix. Returns (ws, b3)."""
    A = np.asarray(A, dtype=np.float64)
    J = np.asarray(J, dtype=np.float64)
    keep = np.max(np.abs(A), axis=1) <= a_fit
    X, Y = windows(A[keep], J[keep], W, a_scale, j_scale)
    Xb = np.hstack([X, np.ones((X.shape[0], 1))])
    G = Xb.T @ Xb
    G = G + lambda_rel * np.trace(G) / G.shape[0] * np.eye(G.shape[0])
    sol = np.linalg.solve(G, Xb.T @ Y)
    return sol[:-1], float(sol[-1])

