"""Pins of the oracle's SCF options that the paper leaves open (Sec. 3.1: the
particle number must stay right during the iteration): the contraction-aware
stopping rule and the particle-number guard."""
import numpy as np
import pytest

import workloads as W
from oracle import scf as SC


def _first_stop(rule, E, tol):
    d = []
    for k in range(1, len(E)):
        d.append(E[k] - E[k - 1])
        if SC.converged_by(rule, d, tol):
            return k
    return None


@pytest.mark.parametrize("rho", [0.3, 0.7, 0.9, 0.97])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_contraction_rule_bounds_the_error_of_a_geometric_tail(rho, sign):
    """E_k = E_inf + c (sign rho)^k: the rule stops only once |E_k - E_inf| < tol.
    For a monotone tail its bound equals the error, so it stops at the first such
    step; for an alternating one the bound exceeds the error by (1 + rho)/(1 - rho)."""
    tol, c, Einf = 1e-6, 0.05, -2.5
    E = [Einf + c * (sign * rho) ** k for k in range(2000)]
    k = _first_stop("contraction", E, tol)
    assert abs(E[k] - Einf) < tol
    slack = 1.0 if sign > 0 else (1.0 + rho) / (1.0 - rho)
    assert abs(E[k - 1] - Einf) * slack >= tol * (1 - 1e-9)     # the bound one step earlier was not met


def test_delta_rule_stops_early_on_a_slow_tail():
    """|dE| < tol alone stops while the error is still rho/(1 - rho) times larger."""
    tol, rho = 1e-6, 0.97
    E = [-1.0 + 0.05 * rho ** k for k in range(3000)]
    k = _first_stop("delta", E, tol)
    err = abs(E[k] + 1.0)
    assert err > 20 * tol and err < 40 * tol


def test_contraction_rule_needs_three_changes_and_a_contraction():
    assert not SC.converged_by("contraction", [1e-9, 1e-10], 1e-6)
    assert not SC.converged_by("contraction", [1e-7, 1e-7, 2e-7], 1e-6)      # growing: rho > 1
    assert SC.converged_by("contraction", [1e-3, 0.0], 1e-6)                   # exact fixed point
    assert SC.converged_by("delta", [1e-7], 1e-6) and not SC.converged_by("delta", [2e-6], 1e-6)


@pytest.fixture(scope="module")
def he():
    return W.he_1d(half_width=6.0, n_e=3, n_g=4, beta=10.0, M=64)


def test_contraction_stop_is_within_tol_of_the_converged_energy(he):
    ref = SC.scf(he, tol=1e-13)
    r = SC.scf(he, tol=1e-6, stop="contraction")
    assert r.converged and abs(r.E - ref.E) < 1e-6
    d = SC.scf(he, tol=1e-6)
    assert r.iters >= d.iters


def test_guard_restarts_a_start_with_the_wrong_electron_count(he):
    """A start holding a quarter of the electrons (N = 0.5 instead of 2) is replaced
    by G0 with alpha halved: the result is the HF-started run at alpha / 2, one
    wasted step ahead of it."""
    setup, hf, G0 = SC.hf_start(he)
    half = SC.scf(he, alpha=0.15, tol=1e-10, setup=setup, hf=hf)
    r = SC.scf(he, alpha=0.3, tol=1e-10, G_init=0.25 * G0, guard=True, setup=setup, hf=hf)
    assert r.backoffs == 1 and r.alpha == 0.15 and r.wasted == 1
    assert r.iters == half.iters + 1
    assert np.max(np.abs(r.G - half.G)) == 0.0 and r.E == half.E
    # without the guard the wrong start is iterated as given
    u = SC.scf(he, alpha=0.3, tol=1e-10, G_init=0.25 * G0, fixed_iters=2, setup=setup, hf=hf)
    assert abs(u.energies[0] - half.energies[0]) > 0.1


def test_guard_gives_up_after_three_restarts(he):
    """A system that keeps failing the guard (here: asking for a particle
    number the HF state does not hold) stops being restarted after three
    halvings and is then iterated with alpha / 8."""
    sysd = he.with_(n_elec=2.0)
    setup, hf, G0 = SC.hf_start(sysd)
    bad = sysd.with_(n_elec=6.0)          # the guard compares N with 6, the state holds 2
    r = SC.scf(bad, alpha=0.4, tol=1e-8, guard=True, setup=setup, hf=hf, max_iter=3)
    assert r.backoffs == 3 and r.alpha == 0.05 and r.wasted == 3
