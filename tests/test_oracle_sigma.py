"""Pins of the oracle's second-Born self-energy (paper Sec. 2.3, Eq. sigma2ndb).

The index reading and the sign are fixed by results that do not come from the
formula itself: the half-filled one-site limit (-U^2/8), and the lowest-order
Galitskii-Migdal energy, which must be twice the textbook closed-shell MP2
energy. The exchange term as printed in the paper fails the second test."""
import numpy as np
import pytest

import workloads as W
from oracle import fedvr, hf as H, sigma as S, ed as ED


def _rand(n, seed):
    V = np.abs(W.random_symmetric(n, seed)) + 0.1
    G = W.random_symmetric(n, seed + 1, 0.3)
    Gb = W.random_symmetric(n, seed + 2, 0.3)
    return V, G, Gb


@pytest.mark.parametrize("n,sigma", [(3, 2), (4, 1), (5, 2)])
def test_three_forms_agree(n, sigma):
    V, G, Gb = _rand(n, 10 * n + sigma)
    a = S.sigma2b_literal(V, G, Gb, sigma)
    b = S.sigma2b_general(S.dvr_eri(V), G, Gb, sigma)
    c = S.sigma2b_slice(V, G, Gb, sigma)
    scale = np.max(np.abs(a))
    assert np.max(np.abs(a - b)) < 1e-13 * scale
    assert np.max(np.abs(a - c)) < 1e-13 * scale


def test_atomic_limit():
    """n_b = 1, V = U, half filling (xi = 0): G0 = -1/2 on (0, beta), and the
    second-order self-energy is -U^2/8 for every tau (sigma = 2); with sigma = 1
    (spinless) it vanishes."""
    U = 1.7
    G = np.array([[-0.5]])
    assert abs(S.sigma2b_literal(np.array([[U]]), G, G, 2)[0, 0] + U * U / 8) < 1e-15
    assert S.sigma2b_literal(np.array([[U]]), G, G, 1)[0, 0] == 0.0


def test_quadratic_in_interaction_and_symmetric():
    V, G, Gb = _rand(6, 3)
    a = S.sigma2b_slice(V, G, Gb, 2)
    b = S.sigma2b_slice(0.3 * V, G, Gb, 2)
    assert np.max(np.abs(b - 0.09 * a)) < 1e-14 * np.max(np.abs(a))
    assert np.max(np.abs(a - a.T)) < 1e-14 * np.max(np.abs(a))


def test_all_slices_pairing():
    V = np.abs(W.random_symmetric(4, 1)) + 0.1
    G = W.random_symmetric_slices(4, 7, 2)
    out = S.sigma2b(V, G, 2)
    for q in range(7):
        assert np.allclose(out[q], S.sigma2b_literal(V, G[q], G[6 - q], 2), rtol=0, atol=1e-13)


def printed_reading(V, G, Gb, sigma):
    """Eq. sigma2ndb with the printed line subscripts u_14 u_23 (V_il V_jk)."""
    d = np.einsum("il,jk,ij,kl,lk->ij", V, V, G, G, Gb)
    x = np.einsum("il,jk,il,kj,lk->ij", V, V, G, G, Gb)
    return sigma * d - x


def gm_correlation_lowest_order(st, hfr, beta, fn, nodes=30, levels=28):
    """-(sigma/2) int_0^beta Tr[Sigma_c[G0](beta - tau) G0(tau)] dtau by composite
    Gauss-Legendre on a geometrically graded partition (G0 exact at every node)."""
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    br = np.array([0.0] + [beta / 2 * 2.0 ** (-k) for k in range(levels, 0, -1)] + [beta / 2])
    full = np.concatenate((br, beta - br[::-1][1:]))
    ts = np.concatenate([0.5 * (b - a) * xg + 0.5 * (a + b) for a, b in zip(full[:-1], full[1:])])
    ws = np.concatenate([0.5 * (b - a) * wg for a, b in zip(full[:-1], full[1:])])
    G = H.g0_tau(hfr, ts)
    Gb = H.g0_tau(hfr, beta - ts)
    tot = 0.0
    for q in range(len(ts)):
        Sc = fn(st.V, Gb[q], G[q], 2)          # Sigma_c(beta - tau): its Gbar is G(tau)
        tot += ws[q] * np.sum(Sc * G[q].T)
    return -tot


@pytest.fixture(scope="module")
def tiny():
    sysd = W.he_1d(half_width=8.0, n_e=4, n_g=4, beta=60.0)
    st = fedvr.Setup(sysd)
    hfr = H.hartree_fock(st.h, st.V, 2.0, 2, 60.0)
    E0, eps0, C0 = ED.rhf_zero_temperature(st.h, st.V, 1)
    return st, hfr, ED.mp2_closed_shell(eps0, C0, st.V, 1)


def test_lowest_order_gm_energy_is_twice_mp2(tiny):
    st, hfr, mp2 = tiny
    e = gm_correlation_lowest_order(st, hfr, 60.0, S.sigma2b_slice)
    assert abs(e / mp2 - 2.0) < 2e-6


def test_printed_exchange_reading_fails_mp2(tiny):
    st, hfr, mp2 = tiny
    e = gm_correlation_lowest_order(st, hfr, 60.0, printed_reading)
    assert abs(e / mp2 - 2.0) > 0.5
