"""Pins of the oracle's tau-convolution quadrature, Dyson step and energy
(paper Sec. 2.3, Eq. deq): exact integrals, closed-form limits, invariants."""
import numpy as np
import pytest

import workloads as W
from oracle import fedvr, hf as H, sigma as S, dyson as D, scf as SC


def _analytic_q(a, b, tau, beta):
    """int_0^beta A(tau - s) B(s) ds for A(x) = e^(-a x) on (0, beta) continued
    antiperiodically, B(s) = e^(-b s)."""
    def seg(lo, hi, c0, rate):          # int_lo^hi c0 e^(rate s) ds
        if abs(rate) < 1e-14:
            return c0 * (hi - lo)
        return c0 * (np.exp(rate * hi) - np.exp(rate * lo)) / rate
    first = seg(0.0, tau, np.exp(-a * tau), a - b)
    second = seg(tau, beta, np.exp(-a * (beta + tau)), a - b)
    return first - second


@pytest.mark.parametrize("a,b", [(1.3, 0.4), (-0.7, 2.0), (2.5, -1.0)])
def test_split_trapezoid_second_order(a, b):
    beta = 4.0
    errs = []
    for M in (64, 128, 256):
        t = fedvr.tau_uniform(beta, M)
        A = np.exp(-a * t)[:, None, None]
        B = np.exp(-b * t)[:, None, None]
        Q = D.conv_direct(lambda p, q, s: D.kernel_grid(A, p, q, s), B, t)[:, 0, 0]
        ex = np.array([_analytic_q(a, b, x, beta) for x in t])
        errs.append(np.max(np.abs(Q - ex)))
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_fft_route_equals_direct():
    n, M = 4, 32
    A = W.random_symmetric_slices(n, M + 1, 5)
    B = W.random_symmetric_slices(n, M + 1, 6)
    t = fedvr.tau_uniform(3.0, M)
    q1 = D.conv_direct(lambda p, q, s: D.kernel_grid(A, p, q, s), B, t)
    q2 = D.conv_uniform_fft(A, B, 3.0 / M)
    assert np.max(np.abs(q1 - q2)) < 1e-13 * np.max(np.abs(q1))
    assert np.max(np.abs(q2[0] + q2[-1])) == 0.0


def test_power_mesh_with_p1_equals_uniform():
    sysu = W.he_1d(half_width=5.0, n_e=3, n_g=4, beta=8.0, M=24)
    sysp = sysu.with_(tau_kind="power", u=12, p=1)
    ru = SC.scf(sysu, fixed_iters=2, route="direct")
    rp = SC.scf(sysp, fixed_iters=2)
    assert np.max(np.abs(ru.G - rp.G)) < 1e-12
    assert abs(ru.E - rp.E) < 1e-12


@pytest.fixture(scope="module")
def he_small():
    sysd = W.he_1d(half_width=6.0, n_e=3, n_g=4, beta=10.0, M=64)
    setup, hf = SC.run_hf(sysd)
    return sysd, setup, hf


def test_fixed_point_without_correlation(he_small):
    sysd, setup, hf = he_small
    ctx = D.DysonContext(setup, hf, "uniform")
    G1 = D.dyson_step(ctx, ctx.G0, np.zeros_like(ctx.G0), 1.0)
    assert np.max(np.abs(G1 - ctx.G0)) < 1e-11


def test_static_perturbation_closed_form():
    """V = 0, Sigma_c = 0 and a static extra term dh (entered as Sigma0 = -dh): the
    Dyson fixed point is the HF-form G of h + dh at the same mu, up to O(dtau^2)."""
    errs = []
    for M in (64, 128):
        sysd = W.he_1d(half_width=5.0, n_e=3, n_g=4, beta=6.0, M=M).with_(ee_scale=0.0)
        setup, hf = SC.run_hf(sysd)
        n = setup.h.shape[0]
        dh = 0.05 * W.random_symmetric(n, 4)
        hf.Sigma0 = -dh
        ctx = D.DysonContext(setup, hf, "uniform")
        G = ctx.G0.copy()
        for _ in range(200):
            Gn = D.dyson_step(ctx, G, np.zeros_like(G), 1.0)
            if np.max(np.abs(Gn - G)) < 1e-14:
                break
            G = Gn
        e2, C2 = np.linalg.eigh(setup.h + dh)
        ref = H.HFResult(e2, C2, hf.mu, None, None, None, 0, 6.0)
        errs.append(np.max(np.abs(G - H.g0_tau(ref, setup.tau))))
    assert errs[0] < 1e-3 and 3.5 < errs[0] / errs[1] < 4.5


def test_jump_condition_every_iterate(he_small):
    sysd, setup, hf = he_small
    ctx = D.DysonContext(setup, hf, "uniform")
    G = ctx.G0
    n = G.shape[1]
    for _ in range(3):
        Sc = S.sigma2b(setup.V, G, 2)
        G = D.dyson_step(ctx, G, Sc, 0.3)
        assert np.max(np.abs(G[0] + G[-1] + np.eye(n))) < 1e-13
        assert np.max(np.abs(G - G.transpose(0, 2, 1))) == 0.0


def test_routes_agree_and_symmetrisation_is_second_order(he_small):
    """The direct and Fourier routes give the same iterates. The left-sided discrete
    Dyson equation has a fixed point that is symmetric only up to O(dtau^2), so
    symmetrising each iterate moves the fixed point by O(dtau^2)."""
    sysd, setup, hf = he_small
    c = SC.scf(sysd, fixed_iters=3, route="direct", setup=setup, hf=hf)
    d = SC.scf(sysd, fixed_iters=3, route="fft", setup=setup, hf=hf)
    assert np.max(np.abs(c.G - d.G)) < 1e-13
    diffs = []
    for M in (64, 128):
        s2 = sysd.with_(M=M)
        a = SC.scf(s2, tol=1e-12)
        b = SC.scf(s2, tol=1e-12, symmetrize=False)
        diffs.append(abs(a.E - b.E))
    assert diffs[0] < 1e-6 and 3.5 < diffs[0] / diffs[1] < 4.5


def test_energy_reduces_to_hf(he_small):
    sysd, setup, hf = he_small
    G0 = H.g0_tau(hf, setup.tau)
    E = D.gm_energy(setup.h, setup.V, 2, G0, np.zeros_like(G0), setup.tau)
    assert abs(E - hf.E) < 1e-13


def test_power_mesh_converges_to_uniform_limit():
    """Fixed-iteration SCF on power meshes of growing u approaches the fine uniform
    result (interpolation O(h^4), trapezoid O(h^2))."""
    base = W.he_1d(half_width=5.0, n_e=3, n_g=4, beta=8.0)
    ref = SC.scf(base.with_(M=512), fixed_iters=2).E
    errs = [abs(SC.scf(base.with_(tau_kind="power", u=u, p=3), fixed_iters=2).E - ref)
            for u in (4, 8)]
    assert errs[1] < errs[0] / 2.5


def _interp_args(t, u):
    """Off-node arguments on a power mesh: random ones, the midpoints of every
    interval, and arguments a hair inside either side of every block boundary
    (node index a multiple of u)."""
    rng = np.random.default_rng(17)
    s = list(rng.uniform(t[0], t[-1], size=200))
    s += list(0.5 * (t[1:] + t[:-1]))
    for b in range(u, len(t) - 1, u):
        for side in (-1, 1):
            h = t[b + side] - t[b] if side > 0 else t[b] - t[b - 1]
            s.append(t[b] + side * 1e-6 * h)
    return np.array(s)


def test_lagrange4_on_power_mesh_is_cubic_exact_with_the_stencil_in_its_block():
    """Reading of the power-mesh convolution (Sigma_c between grid points): 4-point
    Lagrange interpolation inside the uniform block of the argument. Pinned with
    the textbook remainder: for f(x) = (x - s)^4 the interpolant at s equals
    -prod_m (s - t_m) exactly (f'''' = 24), and any cubic is reproduced. The
    stencil is 4 consecutive nodes of the block that holds s and brackets s."""
    u, p, beta = 6, 4, 10.0
    t = fedvr.tau_power(beta, u, p)
    c = np.array([0.7, -1.3, 0.4, 0.05])
    for s in _interp_args(t, u):
        nodes, w = D.lagrange4(t, s, u)
        tn = t[nodes]
        # stencil: consecutive, inside one uniform block, around s
        assert np.all(np.diff(nodes) == 1)
        blk = nodes[0] // u
        assert nodes[-1] <= (blk + 1) * u
        assert t[blk * u] <= s <= t[min((blk + 1) * u, len(t) - 1)]
        assert tn[0] <= s <= tn[3]
        a = int(np.searchsorted(t, s, side="right")) - 1
        if a - 1 >= blk * u and a + 2 <= (blk + 1) * u:
            assert tn[1] <= s <= tn[2]
        # equal spacing inside the stencil (the block is uniform)
        h = np.diff(tn)
        assert np.max(np.abs(h - h[0])) < 1e-12 * h[0]
        # cubic exactness
        f = lambda x: c[0] + x * (c[1] + x * (c[2] + x * c[3]))
        assert abs(w @ f(tn) - f(s)) < 1e-12 * (1.0 + abs(f(s)))
        # the remainder of the quartic (x - s)^4
        q = (tn - s) ** 4
        omega = np.prod(s - tn)
        assert abs(w @ q + omega) < 1e-9 * max(np.max(np.abs(w * q)), 1e-300)


def test_lagrange4_fourth_order_off_node():
    """Interpolating a smooth function off the nodes converges like h^4 (error
    ratio 16 when the block step halves)."""
    beta, p = 6.0, 2
    errs = []
    for u in (8, 16, 32):
        t = fedvr.tau_power(beta, u, p)
        s_all = 0.5 * (t[1:] + t[:-1]) + 0.17 * np.diff(t)
        e = 0.0
        for s in s_all:
            nodes, w = D.lagrange4(t, s, u)
            e = max(e, abs(w @ np.exp(-0.8 * t[nodes]) - np.exp(-0.8 * s)))
        errs.append(e)
    assert 13.0 < errs[0] / errs[1] < 19.0 and 13.0 < errs[1] / errs[2] < 19.0
