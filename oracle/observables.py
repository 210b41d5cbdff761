"""One-electron density of the correlated ground state (paper Sec. 2.3: the
density follows from the Matsubara Green's function at equal times; Sec. 3.2,
Fig. 3b shows it for H3+).

Oracle (test infrastructure only). Plain float64.

With rho = -G(beta^-) per spin and the FE-DVR basis functions chi_a (Sec. 2.1,
Eq. basis: Lobatto shape functions divided by the square root of the summed
GLL weight),
    n(x) = sigma sum_ab chi_a(x) chi_b(x) rho_ab.
At a DVR node x_a only chi_a is non-zero, chi_a(x_a) = 1 / sqrt(W_a), so
n(x_a) = sigma rho_aa / W_a.
"""
from __future__ import annotations

import numpy as np


def density_nodes(G: np.ndarray, W: np.ndarray, sigma: int) -> np.ndarray:
    """n at the DVR nodes from the last slice G(beta^-)."""
    return -sigma * np.diag(G[-1]) / W


def lobatto_shape(xe: np.ndarray, x: float) -> np.ndarray:
    """Values at x of the Lagrange polynomials through the element's GLL nodes xe
    (the Lobatto shape functions f_m of Sec. 2.1: f_m(xe_m') = delta_mm')."""
    f = np.ones(len(xe))
    for m in range(len(xe)):
        for j in range(len(xe)):
            if j != m:
                f[m] *= (x - xe[j]) / (xe[m] - xe[j])
    return f


def density_at(grid, rho: np.ndarray, sigma: int, xs) -> np.ndarray:
    """n(x) at arbitrary points of the box from the per-spin density matrix rho.
    On element e, chi_a(x) = f_m(x) / sqrt(W_a) for the basis functions a = idx[e, m]
    that live on it (the bridge functions continue into the next element); the
    dropped Dirichlet end points contribute nothing."""
    out = np.zeros(len(xs))
    for p, x in enumerate(xs):
        e = int(np.searchsorted(grid.bounds, x, side="right")) - 1
        e = min(max(e, 0), grid.n_e - 1)
        f = lobatto_shape(grid.xe[e], x)
        idx = grid.idx[e]
        chi = np.zeros(grid.n_b)
        for m in range(grid.N + 1):
            if idx[m] >= 0:
                chi[idx[m]] += f[m] / np.sqrt(grid.W[idx[m]])
        out[p] = sigma * chi @ rho @ chi
    return out
