"""Pins of the learned-guess oracle: Chebyshev closed form, gradients against
central finite differences, Adam's first step, and a fit that learns."""
import numpy as np

import workloads as W
from oracle import mlp


def test_chebyshev_closed_form():
    th = np.linspace(0.0, np.pi, 17)
    T = mlp.chebyshev(np.cos(th))
    for k in range(mlp.N_CHEB):
        assert np.max(np.abs(T[:, k] - np.cos(k * th))) < 1e-12


def test_features_layout():
    x = np.linspace(-4, 4, 9)
    v = -1.0 / np.sqrt(x ** 2 + 1)
    tau = np.linspace(0, 10, 5)
    F = mlp.features(x, v, [0.5], [1.5], tau, 10.0, [0, 3], [8, 3], [0, 4])
    assert F.shape == (2, mlp.D_IN)
    assert F[0, 0] == x[0] / 10 and F[0, 1] == x[8] / 10 and F[1, 3] == v[3]
    assert F[0, 4] == 1.0 and F[0, 5] == -1.0 and F[1, 5] == 1.0      # T_0, T_1 at t = -1, +1
    assert F[0, 4 + mlp.N_CHEB] == 1.5 and F[0, 4 + mlp.N_CHEB + 1] == 0.0
    assert F[0, 4 + mlp.N_CHEB + mlp.N_CENT] == 0.05


def test_gradient_against_finite_differences():
    rng = np.random.default_rng(3)
    p = W.mlp_init(mlp.LAYERS, seed=1)
    X = rng.normal(size=(7, mlp.D_IN))
    t = rng.normal(size=7) * 0.1
    y, acts = mlp.forward(p, X)
    L, dy = mlp.mse(y, t)
    g = mlp.backward(p, acts, dy)
    idx = rng.choice(p.size, 40, replace=False)
    idx = np.concatenate([idx, [p.size - 1, mlp.D_IN * mlp.HIDDEN + 3]])
    for k in idx:
        e = 1e-6
        pp = p.copy(); pp[k] += e
        pm = p.copy(); pm[k] -= e
        fd = (mlp.mse(mlp.forward(pp, X)[0], t)[0] - mlp.mse(mlp.forward(pm, X)[0], t)[0]) / (2 * e)
        assert abs(fd - g[k]) < 1e-7 + 1e-5 * abs(fd), k


def test_adam_first_step_is_lr_times_sign():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, p - 0.01 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_training_reduces_loss():
    rng = np.random.default_rng(5)
    p = W.mlp_init(mlp.LAYERS, seed=2)
    X = rng.uniform(-1, 1, size=(256, mlp.D_IN))
    t = 0.3 * np.sin(2 * X[:, 0]) * X[:, 4 + 1]
    m = np.zeros_like(p); v = np.zeros_like(p)
    L0 = mlp.mse(mlp.forward(p, X)[0], t)[0]
    for s in range(1, 201):
        y, acts = mlp.forward(p, X)
        L, dy = mlp.mse(y, t)
        p, m, v = mlp.adam_step(p, mlp.backward(p, acts, dy), m, v, s, 1e-3)
    assert L < 0.1 * L0


def test_envelope_properties():
    """1 at a nucleus; symmetric in (i, j); independent of tau; (1 + D/5)^(-3/2)."""
    x = np.linspace(-10, 10, 41)
    tau = np.linspace(0.0, 20.0, 11)
    c = np.array([-2.0, 3.0])
    ii, jj, qq = np.meshgrid(np.arange(41), np.arange(41), np.arange(11), indexing="ij")
    ii, jj, qq = ii.ravel(), jj.ravel(), qq.ravel()
    e = mlp.envelope(x, c, tau, 20.0, ii, jj, qq)
    assert np.array_equal(e, mlp.envelope(x, c, tau, 20.0, jj, ii, 10 - qq))
    k = int(np.argmin(np.abs(x - 3.0)))
    assert mlp.envelope(x, c, tau, 20.0, [k], [k], [3])[0] == 1.0
    # distance 5 from the nearest nucleus on both indices: (1 + 10/5)^(-3/2) = 3^(-3/2)
    m = int(np.argmin(np.abs(x - 8.0)))
    assert np.isclose(mlp.envelope(x, c, tau, 20.0, [m], [m], [5])[0], 3.0 ** -1.5, rtol=1e-14)
    # no nuclei: distance 0
    assert mlp.envelope(x, [], tau, 20.0, [0], [5], [0])[0] == 1.0
