"""Hartree-Fock self-energy, HF ground state, chemical potential and G0(tau)
(paper Sec. 2.3, Eqs. sigmahf, hamhf, hfgf).

Oracle (test infrastructure only). Plain float64.

Conventions (one spin channel; sigma in {1, 2} is the spin degeneracy):
    G(tau) = -<T psi(tau) psi^dagger(0)>, tau in [0, beta], G(tau - beta) = -G(tau).
    rho = <psi^dagger psi> = G(0^-) = -G(beta^-), the equal-time density matrix.
The paper writes the HF Green's function on the branch tau in [-beta, 0]
(Eq. hfgf) as C f e^(-tau xi) C^T; on [0, beta] the same function is
-C (1 - f) e^(-tau xi) C^T.
"""
from __future__ import annotations

import numpy as np


def sigma_hf(V: np.ndarray, rho: np.ndarray, sigma: int) -> np.ndarray:
    """HF self-energy in the DVR (Eq. sigmahf with g(t, t+) = i rho):
    Sigma_ij = delta_ij sigma sum_k V_ik rho_kk - V_ij rho_ij."""
    return np.diag(sigma * (V @ np.diag(rho))) - V * rho


def fermi(x, beta):
    """f(x) = 1 / (1 + e^(beta x)), written so that no exponent is positive."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    pos = x > 0
    ep = np.exp(-beta * x[pos])
    out[pos] = ep / (1.0 + ep)
    out[~pos] = 1.0 / (1.0 + np.exp(beta * x[~pos]))
    return out


def particle_excess(eps, mu, n_spin, beta):
    """sum_k f(eps_k - mu) - N/sigma, monotone increasing in mu.

    When N/sigma is an integer n the sum is evaluated as
    sum_{k >= n} f(eps_k - mu) - sum_{k < n} f(mu - eps_k) (eps ascending), where
    each term is small inside the gap and is computed to full relative accuracy,
    so that the root is well defined even when both terms are ~e^(-beta gap / 2).
    """
    e = np.sort(eps)
    n = int(round(n_spin))
    if abs(n_spin - n) < 1e-12 and 0 <= n <= len(e):
        return float(np.sum(fermi(e[n:] - mu, beta)) - np.sum(fermi(mu - e[:n], beta)))
    return float(np.sum(fermi(e - mu, beta)) - n_spin)


def chemical_potential(eps, n_spin, beta):
    """mu with sum_k f(eps_k - mu) = N/sigma (Sec. 2.3, normalization of the Fermi
    distribution), by bisection on [min eps - 50/beta, max eps + 50/beta] until the
    bracket stops shrinking; returns the final midpoint."""
    lo = float(np.min(eps)) - 50.0 / beta
    hi = float(np.max(eps)) + 50.0 / beta
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if particle_excess(eps, mid, n_spin, beta) > 0.0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def hf_energy(h, V, rho, sigma):
    """E = sigma (Tr[h rho] + 1/2 Tr[Sigma^HF[rho] rho]); the correlation part is
    added by the Galitskii-Migdal formula in ``dyson``."""
    S = sigma_hf(V, rho, sigma)
    return sigma * (np.sum(h * rho.T) + 0.5 * np.sum(S * rho.T))


class HFResult:
    def __init__(self, eps, C, mu, rho, Sigma0, E, iters, beta):
        self.eps, self.C, self.mu, self.rho = eps, C, mu, rho
        self.Sigma0, self.E, self.iters, self.beta = Sigma0, E, iters, beta
        self.f = fermi(eps - mu, beta)


def hartree_fock(h, V, n_elec, sigma, beta, tol_E=1e-13, tol_rho=1e-12, max_iter=1000):
    """Self-consistent HF ground state (Sec. 2.3, Eq. hamhf).

    Start: rho from the core Hamiltonian h (the paper does not say; this is the
    reading used here). Loop: F = h + Sigma^HF[rho]; F = C diag(eps) C^T; mu by
    bisection; rho' = C f C^T; stop when |dE| < tol_E and max|rho' - rho| < tol_rho.
    Returned: (eps, C) of the last Fock matrix F, Sigma0 = F - h (the HF self-energy
    that generated G0), rho = C f C^T (so that G0(beta^-) = -rho exactly), and
    E = hf_energy(rho).
    """
    n_spin = n_elec / sigma
    eps, C = np.linalg.eigh(h)
    mu = chemical_potential(eps, n_spin, beta)
    rho = (C * fermi(eps - mu, beta)) @ C.T
    E_old = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        Sig = sigma_hf(V, rho, sigma)
        F = h + Sig
        eps, C = np.linalg.eigh(F)
        mu = chemical_potential(eps, n_spin, beta)
        rho_new = (C * fermi(eps - mu, beta)) @ C.T
        E = hf_energy(h, V, rho_new, sigma)
        d = np.max(np.abs(rho_new - rho))
        rho = rho_new
        if abs(E - E_old) < tol_E and d < tol_rho:
            break
        E_old = E
    return HFResult(eps, C, mu, rho, Sig, hf_energy(h, V, rho, sigma), it, beta)


def g0_diag(xi, tau, beta):
    """(1 - f(xi)) e^(-tau xi) for tau in [0, beta], in the form with non-positive
    exponents: e^(-tau xi) / (1 + e^(-beta xi)) for xi >= 0, e^((beta - tau) xi) /
    (1 + e^(beta xi)) otherwise. Shape [len(tau), len(xi)]."""
    xi = np.asarray(xi, dtype=np.float64)[None, :]
    tau = np.asarray(tau, dtype=np.float64)[:, None]
    pos = xi >= 0
    a = np.exp(-tau * np.where(pos, xi, 0.0)) / (1.0 + np.exp(-beta * np.where(pos, xi, 0.0)))
    b = np.exp((beta - tau) * np.where(pos, 0.0, xi)) / (1.0 + np.exp(beta * np.where(pos, 0.0, xi)))
    return np.where(pos, a, b)


def g0_tau(hf: HFResult, tau) -> np.ndarray:
    """HF Matsubara Green's function on [0, beta] (Eq. hfgf, moved to tau > 0):
    G0(tau) = -C diag((1 - f_k) e^(-tau xi_k)) C^T, xi = eps - mu; tau = 0 means 0^+
    and tau = beta means beta^-."""
    g = g0_diag(hf.eps - hf.mu, tau, hf.beta)
    return -np.einsum("ak,qk,bk->qab", hf.C, g, hf.C, optimize=True)
