"""Exact two-electron ground state in the same FE-DVR basis, and closed-shell MP2.

Oracle (test infrastructure only). Plain float64. These stand in for the
paper's few-particle TDSE reference (Sec. 3.1, Sec. 3.2) and serve as pins:
second Born solved self-consistently is exact through second order in the
interaction, so E_2B(lambda) - E_ED(lambda) = O(lambda^3).

Two-electron Hamiltonian on the product grid (a, b) (same DVR rules as the
one-body matrices: kinetic non-diagonal, potential and interaction diagonal,
Eqs. vmat, tmat, umat1):
    H_(ab),(cd) = T_ac d_bd + d_ac T_bd + d_ac d_bd (v_a + v_b + V_ab).
Its lowest eigenvector is spatially symmetric, i.e. the singlet.
"""
from __future__ import annotations

import numpy as np


def two_electron_hamiltonian(T, v, V):
    n = T.shape[0]
    I = np.eye(n)
    H = np.kron(T, I) + np.kron(I, T)
    H += np.diag((v[:, None] + v[None, :] + V).reshape(-1))
    return H


def ed_ground_energy(T, v, V):
    return float(np.linalg.eigvalsh(two_electron_hamiltonian(T, v, V))[0])


def ed_ground_energy_iterative(T, v, V, start=None, tol=1e-11):
    """The same lowest eigenvalue for grids too large for a dense n_b^2 x n_b^2
    matrix: Lanczos (scipy's eigsh) on the operator X -> T X + X T + W o X,
    W_ab = v_a + v_b + V_ab, acting on the two-electron amplitude X_ab.
    ``start`` (optional) is a starting amplitude, e.g. the product of the
    lowest one-electron orbital with itself."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    n = T.shape[0]
    Wd = v[:, None] + v[None, :] + V

    def mv(x):
        X = x.reshape(n, n)
        return (T @ X + X @ T + Wd * X).reshape(-1)

    op = LinearOperator((n * n, n * n), matvec=mv, dtype=np.float64)
    v0 = None if start is None else np.asarray(start, dtype=np.float64).reshape(-1)
    return float(eigsh(op, k=1, which="SA", tol=tol, v0=v0, return_eigenvectors=False)[0])


def mo_eri(C, V):
    """(pq|rs) = sum_ab C_ap C_aq V_ab C_br C_bs for the DVR tensor (aa|bb) = V_ab."""
    P = np.einsum("ap,aq->apq", C, C)
    return np.einsum("apq,ab,brs->pqrs", P, V, P, optimize=True)


def mp2_closed_shell(eps, C, V, n_occ):
    """Textbook closed-shell MP2 (spatial orbitals, real):
    E2 = sum_{ij occ, ab virt} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b)."""
    eri = mo_eri(C, V)
    o = slice(0, n_occ)
    vv = slice(n_occ, len(eps))
    iajb = eri[o, vv, o, vv]
    ibja = iajb.transpose(0, 3, 2, 1)
    eo, ev = eps[o], eps[vv]
    den = eo[:, None, None, None] - ev[None, :, None, None] + eo[None, None, :, None] - ev[None, None, None, :]
    return float(np.sum(iajb * (2.0 * iajb - ibja) / den))


def rhf_zero_temperature(h, V, n_occ, tol=1e-13, max_iter=500):
    """Closed-shell RHF with integer occupations ('direct diagonalisation' HF):
    returns (E_HF, eps, C)."""
    eps, C = np.linalg.eigh(h)
    rho = C[:, :n_occ] @ C[:, :n_occ].T
    E_old = np.inf
    for _ in range(max_iter):
        F = h + np.diag(2.0 * (V @ np.diag(rho))) - V * rho
        eps, C = np.linalg.eigh(F)
        rho_new = C[:, :n_occ] @ C[:, :n_occ].T
        d = np.max(np.abs(rho_new - rho))
        rho = rho_new
        S = np.diag(2.0 * (V @ np.diag(rho))) - V * rho
        E = 2.0 * (np.sum(h * rho) + 0.5 * np.sum(S * rho))
        if abs(E - E_old) < tol and d < 1e-12:
            break
        E_old = E
    return E, eps, C
