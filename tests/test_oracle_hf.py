"""Pins of the oracle's HF ground state, chemical potential and G0(tau)
(paper Sec. 2.3, Eqs. sigmahf, hamhf, hfgf)."""
import numpy as np
import pytest

import workloads as W
from oracle import fedvr, hf as H, ed as ED


@pytest.fixture(scope="module")
def he():
    st = fedvr.Setup(W.config_he())
    return st, H.hartree_fock(st.h, st.V, 2.0, 2, 50.0)


def test_sigma_hf_self_interaction_cancels():
    """One spin-paired site: Sigma^HF = sigma V rho - V rho = V rho (sigma = 2);
    for sigma = 1 the same-spin Hartree and Fock terms cancel exactly."""
    V = np.array([[3.0]])
    rho = np.array([[0.4]])
    assert abs(H.sigma_hf(V, rho, 2)[0, 0] - 1.2) < 1e-15
    assert H.sigma_hf(V, rho, 1)[0, 0] == 0.0


def test_chemical_potential_sum_rule(he):
    st, r = he
    assert abs(np.sum(H.fermi(r.eps - r.mu, 50.0)) - 1.0) < 1e-14
    assert r.eps[0] < r.mu < r.eps[1]
    # midgap to leading order for one occupied level
    assert abs(r.mu - 0.5 * (r.eps[0] + r.eps[1])) < 0.05


def test_chemical_potential_noninteger():
    eps = np.array([-1.0, -0.5, 0.2, 0.9])
    mu = H.chemical_potential(eps, 1.37, 10.0)
    assert abs(np.sum(H.fermi(eps - mu, 10.0)) - 1.37) < 1e-13


def test_hf_noninteracting_limit():
    sysd = W.config_he().with_(ee_scale=0.0)
    st = fedvr.Setup(sysd)
    r = H.hartree_fock(st.h, st.V, 2.0, 2, 200.0)
    e0 = np.linalg.eigvalsh(st.h)[0]
    assert abs(r.E - 2 * e0) < 1e-10


def test_hf_matches_integer_occupation_hf(he):
    st, r = he
    E0, eps0, _ = ED.rhf_zero_temperature(st.h, st.V, 1)
    assert abs(r.E - E0) < 1e-8                      # finite beta: e^(-beta gap / 2) ~ 1e-9
    r2 = H.hartree_fock(st.h, st.V, 2.0, 2, 200.0)
    assert abs(r2.E - E0) < 1e-12
    assert np.max(np.abs(r2.eps - eps0)) < 1e-10


def test_hf_variational_against_ed(he):
    st, r = he
    assert r.E > ED.ed_ground_energy(st.T, st.v, st.V)


def test_hf_fixed_point(he):
    st, r = he
    F = st.h + r.Sigma0
    assert np.max(np.abs(F @ r.C - r.C * r.eps)) < 1e-12
    assert np.max(np.abs(H.sigma_hf(st.V, r.rho, 2) - r.Sigma0)) < 1e-11


def test_g0_jump_sum_rule_symmetry(he):
    st, r = he
    t = fedvr.tau_uniform(50.0, 128)
    G0 = H.g0_tau(r, t)
    n = G0.shape[1]
    assert np.max(np.abs(G0[0] + G0[-1] + np.eye(n))) < 1e-14      # G(0+) + G(beta-) = -1
    assert abs(-2 * np.trace(G0[-1]) - 2.0) < 1e-13                 # -sigma Tr G(beta-) = N
    assert np.max(np.abs(G0[-1] + r.rho)) < 1e-15
    assert np.max(np.abs(G0 - G0.transpose(0, 2, 1))) < 1e-15


def test_g0_equation_of_motion(he):
    """-d/dtau G0 = (F - mu) G0 on (0, beta), by central differences."""
    st, r = he
    F = st.h + r.Sigma0
    for tau in (0.3, 7.0, 25.0, 49.0):
        d = 1e-4
        Gp, Gm, G = H.g0_tau(r, [tau + d, tau - d, tau])
        lhs = -(Gp - Gm) / (2 * d)
        rhs = (F - r.mu * np.eye(len(F))) @ G
        assert np.max(np.abs(lhs - rhs)) < 1e-6 * max(1.0, np.max(np.abs(rhs)))


def test_g0_antiperiodic_paper_branch(he):
    """Eq. hfgf on tau in [-beta, 0]: C f e^(-tau xi) C^T equals -G0(tau + beta)."""
    st, r = he
    xi = r.eps - r.mu
    f = H.fermi(xi, 50.0)
    for tau in (-49.0, -20.0, -0.5):
        g_paper = (r.C * (f * np.exp(-tau * xi))) @ r.C.T
        assert np.max(np.abs(g_paper + H.g0_tau(r, [tau + 50.0])[0])) < 1e-12


def test_g0_no_overflow_large_beta_xi():
    eps = np.array([-30.0, -1.0, 2.0, 400.0])
    g = H.g0_diag(eps - 0.0, np.array([0.0, 1.0, 50.0, 100.0]), 100.0)
    assert np.all(np.isfinite(g)) and np.all(g >= 0) and np.all(g <= 1)


@pytest.mark.slow
def test_paper_hf_limit_case2_grid():
    """Sec. 3.1: E_HF limit = -2.2242096 Ha, reached on the case-II 200 a.u. grid at
    n_b ~ 200-300 (here n_e = 29, n_g = 7, n_b = 202)."""
    sysd = W.he_1d(bounds=W.graded_bounds(100.0, 29), n_g=7, beta=100.0)
    st = fedvr.Setup(sysd)
    r = H.hartree_fock(st.h, st.V, 2.0, 2, 100.0)
    assert abs(r.E - (-2.2242096)) < 5e-7
