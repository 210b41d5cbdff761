"""Learned initial guess: features, a 4-layer tanh MLP, its gradients and Adam.

Oracle (test infrastructure only). Plain float64. The paper has no such
component; it is one of the production patterns added around the method: a
small tau-resolved network maps the one-body potential to a correction of the
HF Green's function, G_init(tau) = G0(tau) + sym(dG(tau)).

Per sample (i, j, tau) the input is
    [x_i/s, x_j/s, v(x_i), v(x_j), T_0(t), ..., T_15(t), Z_1, Z_2, Z_3, X_1/s, X_2/s, X_3/s]
with t = 2 tau / beta - 1, T_k the Chebyshev polynomials (T_0 = 1, T_1 = t,
T_k = 2 t T_(k-1) - T_(k-2)), s = 10, and up to three nuclei (zero-padded).
Network: 26 -> 256 -> 256 -> 256 -> 1, tanh after each hidden layer, output
scaled by a fixed factor (the model predicts dG / out_scale). Parameters are
stored flat in the order W1 (26 x 256, row-major, input-major), b1, W2, b2, W3,
b3, W4 (256 x 1), b4. Loss: mean squared error. Optimiser: Adam.
"""
from __future__ import annotations

import numpy as np

N_CHEB = 16
N_CENT = 3
D_IN = 4 + N_CHEB + 2 * N_CENT
HIDDEN = 256
X_SCALE = 10.0
LAYERS = [(D_IN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, 1)]


def n_params() -> int:
    return sum(a * b + b for a, b in LAYERS)


def unflatten(p):
    out, o = [], 0
    for a, b in LAYERS:
        W = p[o:o + a * b].reshape(a, b)
        o += a * b
        bb = p[o:o + b]
        o += b
        out.append((W, bb))
    return out


def chebyshev(t, K=N_CHEB):
    """T_0 .. T_(K-1) at t by the three-term recurrence; shape [len(t), K]."""
    t = np.asarray(t, dtype=np.float64)
    T = np.zeros((t.size, K))
    T[:, 0] = 1.0
    if K > 1:
        T[:, 1] = t
    for k in range(2, K):
        T[:, k] = 2.0 * t * T[:, k - 1] - T[:, k - 2]
    return T


def features(x, v, centres, charges, tau, beta, ii, jj, qq):
    """Input rows for the samples (ii[s], jj[s], qq[s]) (node, node, tau index)."""
    ii, jj, qq = np.asarray(ii), np.asarray(jj), np.asarray(qq)
    S = ii.size
    F = np.zeros((S, D_IN))
    F[:, 0] = x[ii] / X_SCALE
    F[:, 1] = x[jj] / X_SCALE
    F[:, 2] = v[ii]
    F[:, 3] = v[jj]
    F[:, 4:4 + N_CHEB] = chebyshev(2.0 * np.asarray(tau)[qq] / beta - 1.0)
    Z = np.zeros(N_CENT)
    X = np.zeros(N_CENT)
    Z[:len(charges)] = charges
    X[:len(centres)] = np.asarray(centres) / X_SCALE
    F[:, 4 + N_CHEB:4 + N_CHEB + N_CENT] = Z
    F[:, 4 + N_CHEB + N_CENT:] = X
    return F


ENV_L = 5.0


def envelope(x, centres, tau, beta, ii, jj, qq):
    """Fixed envelope of the learned correction at the samples:
    (1 + (d_i + d_j)/L)^(-3/2), d_i the distance of node i to the nearest nucleus
    (0 without nuclei), L = 5; independent of tau. A design choice of the learned
    guess, not part of the paper's method."""
    x = np.asarray(x, dtype=np.float64)
    c = np.asarray(centres, dtype=np.float64).reshape(-1)
    d = np.min(np.abs(x[:, None] - c[None, :]), axis=1) if c.size else np.zeros_like(x)
    u = 1.0 + (d[np.asarray(ii)] + d[np.asarray(jj)]) / ENV_L
    return u ** -1.5


def forward(p, X):
    """Returns (y [S], cache). Hidden layers h = tanh(a W + b); output y = a W4 + b4."""
    layers = unflatten(p)
    acts = [X]
    a = X
    for li, (W, b) in enumerate(layers):
        z = a @ W + b
        a = np.tanh(z) if li < len(layers) - 1 else z
        acts.append(a)
    return a[:, 0], acts


def backward(p, acts, dy):
    """Gradient of sum_s dy_s y_s with respect to the flat parameters."""
    layers = unflatten(p)
    grads = []
    d = dy[:, None]
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        a_in = acts[li]
        gW = a_in.T @ d
        gb = d.sum(axis=0)
        grads.append((gW, gb))
        if li > 0:
            d = (d @ W.T) * (1.0 - acts[li] ** 2)
    grads.reverse()
    return np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])


def mse(y, t):
    r = y - t
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1); step counts from 1. Returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
