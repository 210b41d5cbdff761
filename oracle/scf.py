"""Self-consistent second-Born ground state (paper Sec. 2.3: HF start, Eq. deq
iterated to self-consistency, total energy).

Oracle (test infrastructure only). Plain float64.

Loop (readings: start from G0, linear mixing, symmetrisation, energy of the
Green's function that enters each iteration; the paper fixes none of these):
    k = 0, 1, ...:  Sc_k = Sigma_c[G_k];  E_k = E_GM[G_k, Sc_k]
                    stop if k >= 1 and |E_k - E_{k-1}| < tol  (return G_k, E_k)
                    G_{k+1} = dyson_step(G_k, Sc_k)
With ``fixed_iters = K`` the loop runs exactly K Dyson steps and returns G_K, E_K.

Two options of this build (readings, not in the paper), applied identically by
the library:
  stop="contraction": stop when the geometric tail bound of the energy error,
      |d_k| rho / (1 - rho) with d_k = E_k - E_(k-1) and rho the larger of the
      last two ratios |d_k / d_(k-1)|, |d_(k-1) / d_(k-2)|, is below tol
      (k >= 3; rho < 1; d_k = 0 also stops). stop="delta" is |d_k| < tol.
  guard=True: a run that leaves the iteration's basin restarts from G0 with
      half the mixing parameter, at most three times; the steps before a
      restart are counted in ``iters`` and listed in ``wasted``. Signs of a
      runaway: E_k or N_k not finite, the particle number off by more than a
      half (|N_k - N| > N/2; Sec. 3.1 asks for a stable N), or the energy
      change growing three times in a row (|d_k| > |d_(k-1)| > |d_(k-2)| > |d_(k-3)|).
      A converged fixed point whose N differs from N by less than that is
      accepted: the chemical potential stays at its HF value.
"""
from __future__ import annotations

import numpy as np

from .fedvr import Setup
from .hf import hartree_fock, g0_tau
from .sigma import sigma2b
from .dyson import DysonContext, dyson_step, gm_energy, particle_number


class SCFResult:
    def __init__(self, G, E, N, iters, converged, energies, hf, setup):
        self.G, self.E, self.N, self.iters = G, E, N, iters
        self.converged, self.energies, self.hf, self.setup = converged, energies, hf, setup


def run_hf(sysd, setup=None):
    setup = Setup(sysd) if setup is None else setup
    hf = hartree_fock(setup.h, setup.V, sysd.n_elec, sysd.sigma, sysd.beta)
    return setup, hf


N_GUARD = 0.5           # relative particle-number drift that triggers a restart
MAX_BACKOFF = 3         # restarts with halved mixing


def runaway(E, N, n_elec, d):
    """The guard's test on the energy E_k, particle number N_k and the energy
    changes d of the current run (d_k last)."""
    if not (np.isfinite(E) and np.isfinite(N)):
        return True
    if abs(N - n_elec) > N_GUARD * n_elec:
        return True
    return len(d) >= 4 and abs(d[-1]) > abs(d[-2]) > abs(d[-3]) > abs(d[-4])


def converged_by(rule, d, tol):
    """The stopping test on the energy changes d = [d_1, ..., d_k] of the current run."""
    if not d:
        return False
    if rule == "delta":
        return abs(d[-1]) < tol
    if abs(d[-1]) == 0.0:
        return True
    if len(d) < 3 or d[-2] == 0.0 or d[-3] == 0.0:
        return False
    rho = max(abs(d[-1] / d[-2]), abs(d[-2] / d[-3]))
    return rho < 1.0 and abs(d[-1]) * rho / (1.0 - rho) < tol


def scf(sysd, alpha=0.3, tol=1e-8, max_iter=1000, route="fft", symmetrize=True,
        G_init=None, fixed_iters=None, setup=None, hf=None, stop="delta", guard=False):
    if setup is None or hf is None:
        setup, hf = run_hf(sysd, setup)
    block = sysd.u if sysd.tau_kind == "power" else 0
    ctx = DysonContext(setup, hf, sysd.tau_kind, block)
    G = ctx.G0.copy() if G_init is None else np.array(G_init, dtype=np.float64)
    energies = []
    converged = False
    limit = fixed_iters if fixed_iters is not None else max_iter
    k = 0
    d = []                  # energy changes of the current run
    wasted = 0
    backoffs = 0
    while True:
        Sc = sigma2b(setup.V, G, sysd.sigma)
        E = gm_energy(setup.h, setup.V, sysd.sigma, G, Sc, setup.tau, sysd.e_nn)
        N = particle_number(G, sysd.sigma)
        energies.append(E)
        if k >= 1:
            d.append(E - energies[-2])
        if guard and backoffs < MAX_BACKOFF and runaway(E, N, sysd.n_elec, d):
            wasted += k + 1
            backoffs += 1
            alpha *= 0.5
            G = ctx.G0.copy()
            k = 0
            d = []
            continue
        if fixed_iters is None and converged_by(stop, d, tol):
            converged = True
            break
        if k >= limit:
            break
        G = dyson_step(ctx, G, Sc, alpha, symmetrize, route)
        k += 1
    r = SCFResult(G, E, particle_number(G, sysd.sigma), wasted + k, converged, energies, hf, setup)
    r.wasted, r.alpha, r.backoffs = wasted, alpha, backoffs
    return r


def hf_start(sysd, setup=None):
    setup, hf = run_hf(sysd, setup)
    return setup, hf, g0_tau(hf, setup.tau)
