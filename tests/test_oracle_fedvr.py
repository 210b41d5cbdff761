"""Pins of the oracle's FE-DVR grid and matrices (paper Sec. 2.1-2.2) against
quadrature theory, closed forms and textbook spectra."""
import numpy as np
import pytest

import workloads as W
from oracle import fedvr


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 7, 10, 15])
def test_gll_exact_to_degree_2N_minus_1(N):
    x, w = fedvr.gll_points(N)
    assert len(x) == N + 1
    for k in range(2 * N):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** k) - exact) < 1e-13
    k = 2 * N
    assert abs(np.sum(w * x ** k) - 2.0 / (k + 1)) > 1e-11     # not exact one degree higher


def test_gll_closed_forms():
    x, w = fedvr.gll_points(4)
    assert np.allclose(x, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], atol=1e-15)
    assert np.allclose(w, [0.1, 49 / 90, 32 / 45, 49 / 90, 0.1], atol=1e-15)
    x, w = fedvr.gll_points(5)
    a = np.sqrt(1 / 3 - 2 * np.sqrt(7) / 21)
    b = np.sqrt(1 / 3 + 2 * np.sqrt(7) / 21)
    assert np.allclose(x, [-1, -b, -a, a, b, 1], atol=1e-15)
    assert np.allclose(w, [1 / 15, (14 - np.sqrt(7)) / 30, (14 + np.sqrt(7)) / 30,
                           (14 + np.sqrt(7)) / 30, (14 - np.sqrt(7)) / 30, 1 / 15], atol=1e-15)
    x, w = fedvr.gll_points(6)
    a = np.sqrt(5 / 11 - 2 / 11 * np.sqrt(5 / 3))
    b = np.sqrt(5 / 11 + 2 / 11 * np.sqrt(5 / 3))
    assert np.allclose(x, [-1, -b, -a, 0, a, b, 1], atol=1e-15)
    assert np.allclose(w[[0, 1, 2, 3]], [1 / 21, (124 - 7 * np.sqrt(15)) / 350,
                                         (124 + 7 * np.sqrt(15)) / 350, 256 / 525], atol=1e-15)


@pytest.mark.parametrize("N", [3, 5, 8])
def test_derivative_matrix_exact_on_polynomials(N):
    x, _ = fedvr.gll_points(N)
    D = fedvr.lagrange_derivative_matrix(x)
    for k in range(N + 1):
        want = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        assert np.max(np.abs(D @ x ** k - want)) < 1e-12
    # closed-form corner entries
    assert abs(D[0, 0] + N * (N + 1) / 4) < 1e-12
    assert abs(D[N, N] - N * (N + 1) / 4) < 1e-12


def test_basis_dimension_and_paper_counts():
    assert W.config_he().n_b == 19
    assert W.config_sigma_bench().n_b == 199
    assert W.config_h3p().n_b == 359
    assert fedvr.Grid(W.graded_bounds(100.0, 29), 7).n_b == 202     # Sec. 3.1, n_e = 29, n_g = 7
    assert fedvr.Grid(W.graded_bounds(25.0, 13), 11).n_b == 142     # Sec. 3.2, n_e = 13
    g = fedvr.Grid(W.uniform_bounds(5.0, 3), 4)
    assert np.all(np.diff(g.x) > 0) and g.n_b == 11


def test_quadrature_integrates_polynomials_on_the_grid():
    g = fedvr.Grid(W.uniform_bounds(3.0, 5), 6)
    # sum_a W_a p(x_a) = int p over the box minus the two dropped end-node terms
    xg, wg = fedvr.gll_points(6)
    h = 6.0 / 5
    ends = 0.5 * h * wg[0]
    for k in range(0, 12, 2):
        exact = 2 * 3.0 ** (k + 1) / (k + 1)
        got = np.sum(g.W * g.x ** k) + ends * (3.0 ** k + 3.0 ** k)
        assert abs(got - exact) < 1e-11 * max(1, exact)


def _setup(L, n_e, N):
    return fedvr.Setup(W.he_1d(half_width=L, n_e=n_e, n_g=N))


def test_kinetic_symmetric_banded():
    st = _setup(10.0, 6, 5)
    T = st.T
    assert np.max(np.abs(T - T.T)) < 1e-13
    assert np.all(np.linalg.eigvalsh(T) > 0)
    n = T.shape[0]
    for i in range(n):
        for j in range(n):
            if abs(i - j) > 5:
                assert T[i, j] == 0.0


def test_kinetic_particle_in_a_box():
    st = _setup(10.0, 10, 8)
    ev = np.linalg.eigvalsh(st.T)[:5]
    ref = np.array([(k * np.pi / 20.0) ** 2 / 2 for k in range(1, 6)])
    assert np.max(np.abs(ev - ref) / ref) < 1e-10


def test_harmonic_oscillator_spectrum():
    st = _setup(10.0, 12, 8)
    ev = np.linalg.eigvalsh(st.T + np.diag(st.x ** 2 / 2))[:4]
    assert np.max(np.abs(ev - (np.arange(4) + 0.5))) < 1e-6


def test_soft_core_hydrogen_matches_h3p_threshold():
    """The paper's H3+ dissociation threshold -1.3396 Ha is twice the 1D soft-core
    hydrogen ground state (Sec. 3.2)."""
    st = _setup(25.0, 25, 8)
    e = np.linalg.eigvalsh(st.T - np.diag(1.0 / np.sqrt(st.x ** 2 + 1)))[0]
    assert abs(2 * e - (-1.3396)) < 1e-4


def test_spectral_convergence_in_N():
    errs = []
    for N in (3, 5, 7):
        st = _setup(10.0, 8, N)
        e = np.linalg.eigvalsh(st.T + np.diag(st.x ** 2 / 2))[0]
        errs.append(abs(e - 0.5))
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10


def test_interaction_eigen_route_equals_direct():
    st = _setup(6.0, 4, 5)
    Ve = fedvr.interaction_eigen_route(st.grid)
    assert np.max(np.abs(Ve - st.V)) < 1e-12
    b = W.graded_bounds(10.0, 5)
    g = fedvr.Grid(b, 4)
    assert np.max(np.abs(fedvr.interaction_eigen_route(g) - fedvr.interaction_direct(g.x))) < 1e-12


def test_tau_grids():
    t = fedvr.tau_uniform(50.0, 128)
    assert len(t) == 129 and t[0] == 0.0 and t[-1] == 50.0
    assert np.all(t + t[::-1] == 50.0)
    assert np.max(np.abs(np.diff(t) - 50.0 / 128)) < 1e-13
    tp = fedvr.tau_power(100.0, 64, 16)
    assert len(tp) == 2 * 64 * 16 + 1 == 2049
    assert np.all(tp + tp[::-1] == 100.0) and np.all(np.diff(tp) > 0)
    d = np.diff(tp)
    assert abs(d.min() - 100.0 / 2 ** 16 / 64) < 1e-15
    assert abs(d.max() - 100.0 / 4 / 64) < 1e-12
    # p = 1 is the uniform grid with 2u intervals
    assert np.max(np.abs(fedvr.tau_power(10.0, 8, 1) - fedvr.tau_uniform(10.0, 16))) < 1e-14


def test_graded_layout():
    b = W.graded_bounds(100.0, 29)
    w = np.diff(b)
    assert abs(w[14] - 1.0) < 1e-14 and abs(b[0] + 100) < 1e-12 and abs(b[-1] - 100) < 1e-12
    assert np.allclose(w, w[::-1]) and np.all(np.diff(w[14:]) > 0)
