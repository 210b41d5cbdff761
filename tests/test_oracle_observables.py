"""Pins of the oracle's density n(x) (paper Sec. 2.3: density from the equal-time
Green's function; Fig. 3b) and of the harmonic-trap potential (the paper's
conclusion: fermions in a harmonic trap)."""
import numpy as np
import pytest

import workloads as W
from oracle import fedvr, hf as H, observables as O, scf as SC


def _trap(n_elec, ee, half_width=8.0, n_e=16, n_g=8, beta=40.0):
    return W.harmonic_trap(n_elec=n_elec, omega=1.0, half_width=half_width, n_e=n_e, n_g=n_g, beta=beta, M=64,
                           ee_scale=ee)


def test_harmonic_oscillator_density_is_the_textbook_gaussian():
    """Two non-interacting electrons in (1/2) x^2 fill the oscillator ground state:
    n(x) = 2 e^(-x^2) / sqrt(pi), here tested at points between the DVR nodes."""
    s = _trap(2.0, 0.0)
    st = fedvr.Setup(s)
    r = H.hartree_fock(st.h, st.V, 2.0, 2, s.beta)
    e = np.linalg.eigvalsh(st.h)
    assert np.max(np.abs(e[:4] - (np.arange(4) + 0.5))) < 1e-9
    xs = np.linspace(-3.7, 3.9, 41) + 0.013
    n = O.density_at(st.grid, r.rho, 2, xs)
    assert np.max(np.abs(n - 2.0 * np.exp(-xs ** 2) / np.sqrt(np.pi))) < 1e-7


def test_density_at_the_nodes_and_its_sum_rule():
    s = W.config_he()
    res = SC.scf(s, fixed_iters=3)
    st = res.setup
    nn = O.density_nodes(res.G, st.W, 2)
    assert abs(np.sum(st.W * nn) - res.N) < 1e-12          # sum_a W_a n(x_a) = N (GLL quadrature)
    assert np.max(np.abs(O.density_at(st.grid, -res.G[-1], 2, st.x) - nn)) < 1e-12 * np.max(nn)


def test_density_is_continuous_across_element_boundaries():
    s = W.config_he()
    st = fedvr.Setup(s)
    r = H.hartree_fock(st.h, st.V, 2.0, 2, s.beta)
    for b in st.grid.bounds[1:-1]:
        lo, hi = O.density_at(st.grid, r.rho, 2, [b - 1e-9, b + 1e-9])
        assert abs(lo - hi) < 1e-7 * max(abs(lo), 1e-3)


def test_interacting_trap_density_is_symmetric_and_holds_n():
    s = _trap(4.0, 0.5, n_e=8, n_g=6)
    res = SC.scf(s, fixed_iters=2)
    st = res.setup
    nn = O.density_nodes(res.G, st.W, 2)
    assert np.max(np.abs(nn - nn[::-1])) < 1e-10 * np.max(nn)
    assert abs(np.sum(st.W * nn) - res.N) < 1e-12 and abs(res.N - 4.0) < 1e-3
