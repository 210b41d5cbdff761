"""Second-Born correlation self-energy on the Matsubara grid (paper Sec. 2.3,
Eq. sigma2ndb).

Oracle (test infrastructure only). Plain float64.

For tau in [0, beta] with Gb = G(beta - tau):

    Sigma_c,ij(tau) = sum_kl V_ik V_jl [ sigma G_ij G_kl Gb_lk  -  G_il Gb_lk G_kj ]

Reading of the printed equation: the two interaction lines of each diagram are
taken between points at equal times, V_ik at the outer time and V_jl at the
inner one. The printed subscripts (u_14 u_23) tie the exchange term's lines
to points at different times; with symmetric G the direct term is the same in
both readings and only the exchange term differs. The reading here is the one
Wick's theorem gives for the point-diagonal interaction of Eq. umat1, and the
tests pin it against textbook MP2 and exact diagonalisation. The overall sign
follows from the Matsubara convention G = -<T psi psi^dagger>: in the one-site
half-filled limit it gives Sigma_c = -U^2/8, the second-order atomic result.

Three implementations are kept:
    sigma2b_literal   the four-fold sum as written (tiny n_b only)
    sigma2b_general   the general-basis O(n_b^6) form with the 4-index tensor
                      (ab|cd) = delta_ab delta_cd V_ac inserted (Sec. 2.3: the
                      FE-DVR reduction from O(n_b^6) to O(n_b^2) per element)
    sigma2b_slice     the same sums in optimal order, O(n_b^4) per slice
"""
from __future__ import annotations

import numpy as np


def sigma2b_literal(V, G, Gb, sigma):
    """Four nested loops over i, j, k, l."""
    n = V.shape[0]
    S = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for k in range(n):
                for l in range(n):
                    acc += V[i, k] * V[j, l] * (sigma * G[i, j] * G[k, l] * Gb[l, k]
                                                - G[i, l] * Gb[l, k] * G[k, j])
            S[i, j] = acc
    return S


def dvr_eri(V):
    """Chemist-notation two-electron tensor of the DVR, (ab|cd) = delta_ab delta_cd V_ac
    (Eq. umat1)."""
    n = V.shape[0]
    u = np.zeros((n, n, n, n))
    for a in range(n):
        for c in range(n):
            u[a, a, c, c] = V[a, c]
    return u


def sigma2b_general(eri, G, Gb, sigma):
    """General-basis second Born with a full tensor (ia|cd):
    Sigma_ij = sum_abcdef (ia|cd)(bj|ef) [sigma G_ab G_de Gb_fc - G_ae Gb_fc G_db]."""
    d = np.einsum("iacd,bjef,ab,de,fc->ij", eri, eri, G, G, Gb, optimize=True)
    x = np.einsum("iacd,bjef,ae,fc,db->ij", eri, eri, G, Gb, G, optimize=True)
    return sigma * d - x


def sigma2b_slice(V, G, Gb, sigma):
    """Optimal-order form for one slice.

    direct:   sigma * G o (V (G o Gb^T) V)            (two matrix products)
    exchange: M^(i) = Gb diag(V_i,:) G,  X_ij = sum_l G_il V_jl M^(i)_lj
    """
    D = V @ (G * Gb.T) @ V
    Mx = np.einsum("lk,ik,kj->ilj", Gb, V, G, optimize=True)
    X = np.einsum("il,jl,ilj->ij", G, V, Mx, optimize=True)
    return sigma * G * D - X


def sigma2b(V, G, sigma, slices=None):
    """Sigma_c for every stored tau slice of G [n_tau][n_b][n_b] on a grid symmetric
    under tau -> beta - tau (slot q pairs with slot n_tau - 1 - q).
    ``slices`` restricts the output to the listed slots (others stay zero)."""
    n_tau = G.shape[0]
    out = np.zeros_like(G)
    qs = range(n_tau) if slices is None else slices
    for q in qs:
        out[q] = sigma2b_slice(V, G[q], G[n_tau - 1 - q], sigma)
    return out
