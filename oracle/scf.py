"""Self-consistent second-Born ground state (paper Sec. 2.3: HF start, Eq. deq
iterated to self-consistency, total energy).

Oracle (test infrastructure only). Plain float64.

Loop (readings: start from G0, linear mixing, symmetrisation, energy of the
Green's function that enters each iteration; the paper fixes none of these):
    k = 0, 1, ...:  Sc_k = Sigma_c[G_k];  E_k = E_GM[G_k, Sc_k]
                    stop if k >= 1 and |E_k - E_{k-1}| < tol  (return G_k, E_k)
                    G_{k+1} = dyson_step(G_k, Sc_k)
With ``fixed_iters = K`` the loop runs exactly K Dyson steps and returns G_K, E_K.
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


def scf(sysd, alpha=0.3, tol=1e-8, max_iter=1000, route="fft", symmetrize=True,
        G_init=None, fixed_iters=None, setup=None, hf=None):
    if setup is None or hf is None:
        setup, hf = run_hf(sysd, setup)
    block = sysd.u if sysd.tau_kind == "power" else 0
    ctx = DysonContext(setup, hf, sysd.tau_kind, block)
    G = ctx.G0.copy() if G_init is None else np.array(G_init, dtype=np.float64)
    energies = []
    converged = False
    limit = fixed_iters if fixed_iters is not None else max_iter
    k = 0
    while True:
        Sc = sigma2b(setup.V, G, sysd.sigma)
        E = gm_energy(setup.h, setup.V, sysd.sigma, G, Sc, setup.tau, sysd.e_nn)
        energies.append(E)
        if fixed_iters is None and k >= 1 and abs(E - energies[-2]) < tol:
            converged = True
            break
        if k >= limit:
            break
        G = dyson_step(ctx, G, Sc, alpha, symmetrize, route)
        k += 1
    return SCFResult(G, E, particle_number(G, sysd.sigma), k, converged, energies, hf, setup)


def hf_start(sysd, setup=None):
    setup, hf = run_hf(sysd, setup)
    return setup, hf, g0_tau(hf, setup.tau)
