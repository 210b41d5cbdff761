"""GPU parity of the learned-guess kernels against the float64 oracle
(features, forward pass, gradients, Adam update, full-grid guess).
The network runs in float32; tolerances are float32-level."""
import numpy as np
import pytest

import paper_0911_4348_amd as negf
import workloads as W
from oracle import fedvr, mlp, hf as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = negf.Context(0)
    yield torch, ctx
    ctx.close()


def _sys():
    return W.random_potential_system(7, base=W.he_1d(half_width=8.0, n_e=5, n_g=4, beta=20.0, M=32))


def test_param_count(env):
    assert negf.mlp_param_count() == mlp.n_params()


def test_features_match_oracle(env):
    torch, ctx = env
    s = _sys()
    st = fedvr.Setup(s)
    rng = np.random.default_rng(1)
    S = 300
    ii = rng.integers(0, s.n_b, S)
    jj = rng.integers(0, s.n_b, S)
    qq = rng.integers(0, s.n_tau, S)
    ref = mlp.features(st.x, st.v, s.centres, s.charges, st.tau, s.beta, ii, jj, qq)
    d = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    F = negf.mlp_features(ctx, s, d(st.x, torch.float64), d(st.v, torch.float64), d(st.tau, torch.float64),
                          d(ii, torch.int32), d(jj, torch.int32), d(qq, torch.int32))
    assert np.max(np.abs(F.cpu().numpy() - ref)) < 2e-6


def test_forward_gradient_adam_match_oracle(env):
    torch, ctx = env
    rng = np.random.default_rng(4)
    p = W.mlp_init(mlp.LAYERS, seed=3)
    S = 777
    X = rng.uniform(-1, 1, size=(S, mlp.D_IN))
    t = 0.2 * rng.normal(size=S)
    y_ref, acts = mlp.forward(p, X)
    L_ref, dy = mlp.mse(y_ref, t)
    g_ref = mlp.backward(p, acts, dy)
    p1_ref, m1, v1 = mlp.adam_step(p, g_ref, np.zeros_like(p), np.zeros_like(p), 1, 1e-3)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    P = f32(p)
    y = negf.mlp_forward(ctx, P, f32(X)).cpu().numpy()
    assert np.max(np.abs(y - y_ref)) < 1e-5 * max(1, np.max(np.abs(y_ref)))
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    g = torch.empty_like(P)
    L = negf.mlp_train_step(ctx, P, m, v, 1, 1e-3, f32(X), f32(t), grad_out=g)
    assert abs(L - L_ref) < 1e-5 * L_ref
    gg = g.cpu().numpy()
    assert np.max(np.abs(gg - g_ref)) < 1e-4 * np.max(np.abs(g_ref))
    # the Adam step moves each parameter by ~lr sign(g); compare where g is not tiny
    big = np.abs(g_ref) > 1e-3 * np.max(np.abs(g_ref))
    assert np.max(np.abs(P.cpu().numpy()[big] - p1_ref[big])) < 1e-6


def test_guess_matches_oracle(env):
    torch, ctx = env
    s = _sys()
    st = fedvr.Setup(s)
    hfr = H.hartree_fock(st.h, st.V, 2.0, 2, s.beta)
    G0 = H.g0_tau(hfr, st.tau)
    p = W.mlp_init(mlp.LAYERS, seed=5)
    scale = 0.01
    n = s.n_b
    iu = np.triu_indices(n)
    qq = np.repeat(np.arange(s.n_tau), len(iu[0]))
    ii = np.tile(iu[0], s.n_tau)
    jj = np.tile(iu[1], s.n_tau)
    y, _ = mlp.forward(p, mlp.features(st.x, st.v, s.centres, s.charges, st.tau, s.beta, ii, jj, qq))
    y = y * mlp.envelope(st.x, s.centres, st.tau, s.beta, ii, jj, qq)
    ref = G0.copy()
    dG = np.zeros_like(G0)
    dG[qq, ii, jj] = y * scale
    dG[qq, jj, ii] = y * scale
    ref = 0.5 * (G0 + G0.transpose(0, 2, 1)) + dG
    d64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    out = negf.mlp_guess(ctx, torch.from_numpy(p.astype(np.float32)).cuda(), scale, s, d64(st.x), d64(st.v),
                         d64(st.tau), d64(G0))
    o = out.cpu().numpy()
    assert np.max(np.abs(o - ref)) < 1e-6 * scale * 10 + 1e-12
    assert np.array_equal(o, o.transpose(0, 2, 1))
    # bf16 inference on the matrix cores: the correction within a few percent of its size
    ob = negf.mlp_guess(ctx, torch.from_numpy(p.astype(np.float32)).cuda(), scale, s, d64(st.x), d64(st.v),
                        d64(st.tau), d64(G0), dtype="bf16").cpu().numpy()
    corr = ref - 0.5 * (G0 + G0.transpose(0, 2, 1))
    assert np.max(np.abs(ob - ref)) < 3e-2 * np.max(np.abs(corr))
    assert np.array_equal(ob, ob.transpose(0, 2, 1))


def test_targets_and_envelope_match_oracle(env):
    """Training targets (G - G0) / (scale e) and the envelope at seeded samples."""
    torch, ctx = env
    s = _sys()
    st = fedvr.Setup(s)
    rng = np.random.default_rng(3)
    G = W.random_symmetric_slices(s.n_b, s.n_tau, 21)
    G0 = W.random_symmetric_slices(s.n_b, s.n_tau, 22)
    S = 777
    ii = rng.integers(0, s.n_b, S).astype(np.int32)
    jj = rng.integers(0, s.n_b, S).astype(np.int32)
    qq = rng.integers(0, s.n_tau, S).astype(np.int32)
    e_ref = mlp.envelope(st.x, s.centres, st.tau, s.beta, ii, jj, qq)
    d64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    di = lambda a: torch.from_numpy(a).cuda()
    e = negf.mlp_envelope(ctx, s, d64(st.x), d64(st.tau), di(ii), di(jj), di(qq)).cpu().numpy()
    assert np.max(np.abs(e - e_ref) / e_ref) < 1e-6
    t = negf.mlp_targets(ctx, s, d64(st.x), d64(st.tau), d64(G), d64(G0), 0.5, di(ii), di(jj), di(qq))
    t_ref = (G[qq, ii, jj] - G0[qq, ii, jj]) / (0.5 * e_ref)
    assert np.max(np.abs(t.cpu().numpy() - t_ref)) < 1e-6 * np.max(np.abs(t_ref))
