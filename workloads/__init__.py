"""Seeded synthetic inputs for the FE-DVR second-Born ground-state path.

This module defines inputs only: element boundaries, nuclear centres and
charges, the parameters of the imaginary-time grid, and seeded random arrays.
It holds none of the method's arithmetic (no quadrature rule, no matrix
element, no self-energy, no Dyson step). Both the CPU oracle and the HIP path
consume what it returns, which is the only thing the two share.

Model systems follow the paper's Sec. 3: the soft-Coulomb 1D helium atom
(Sec. 3.1) and the linear 1D H3+ ion (Sec. 3.2, Eq. h3pv), with the
interaction u(|x-x'|) = [(x-x')^2 + 1]^(-1/2) of Sec. 3.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List

import numpy as np


@dataclass
class System:
    """One closed-shell 1D model: grid, potential, interaction, temperature, tau grid.

    ``n_g`` is the number of basis functions per finite element, i.e. the
    number of generalized Gauss-Lobatto points per element minus one, so that
    the basis size is n_b = n_e * n_g - 1 (Sec. 2.1, Eq. basisdim).
    The one-body potential is v(x) = -sum_c Z_c / sqrt((x - X_c)^2 + soft).
    The interaction is V(x, x') = ee_scale / sqrt((x - x')^2 + ee_soft).
    ``tau_kind`` is "uniform" (M intervals, M + 1 points) or "power"
    (2 u p + 1 points clustered at both ends of [0, beta]).
    ``e_nn`` is a constant added once to the total energy (nuclear repulsion).
    ``omega`` > 0 adds a harmonic confinement (1/2) omega^2 x^2 to v.
    """

    name: str
    bounds: np.ndarray
    n_g: int
    centres: np.ndarray
    charges: np.ndarray
    soft: float = 1.0
    ee_soft: float = 1.0
    ee_scale: float = 1.0
    n_elec: float = 2.0
    sigma: int = 2
    beta: float = 50.0
    tau_kind: str = "uniform"
    M: int = 128
    u: int = 0
    p: int = 0
    e_nn: float = 0.0
    omega: float = 0.0

    @property
    def n_e(self) -> int:
        return len(self.bounds) - 1

    @property
    def n_b(self) -> int:
        return self.n_e * self.n_g - 1

    @property
    def n_tau(self) -> int:
        """Number of stored tau points."""
        if self.tau_kind == "uniform":
            return self.M + 1
        return 2 * self.u * self.p + 1

    def with_(self, **kw) -> "System":
        return replace(self, **kw)


# ---------------------------------------------------------------- element layouts

def uniform_bounds(half_width: float, n_e: int) -> np.ndarray:
    """Equidistant finite elements on [-L, L] (the paper's 'case I')."""
    return np.linspace(-half_width, half_width, n_e + 1)


def graded_bounds(half_width: float, n_e: int) -> np.ndarray:
    """Centre element of width 1 a.u., neighbours growing linearly outwards.

    This is the paper's 'case II' layout (Sec. 3.1). The paper does not give the
    growth rule; the widths used here are 1 + k*delta for k = 1 .. (n_e-1)/2 on
    each side, with delta fixed by the box size. n_e must be odd.
    """
    if n_e % 2 != 1:
        raise ValueError("graded layout needs an odd number of elements")
    K = (n_e - 1) // 2
    if K == 0:
        return np.array([-half_width, half_width])
    delta = (2.0 * half_width - 1.0 - 2.0 * K) / (K * (K + 1))
    right = [0.5]
    for k in range(1, K + 1):
        right.append(right[-1] + 1.0 + k * delta)
    right[-1] = half_width
    right = np.array(right)
    return np.concatenate((-right[::-1], right))


# ---------------------------------------------------------------- model systems

def he_1d(half_width=10.0, n_e=4, n_g=5, beta=50.0, M=128, bounds=None) -> System:
    """1D helium: Z = 2 at the origin, softening rho = 1 (Sec. 3.1)."""
    b = uniform_bounds(half_width, n_e) if bounds is None else np.asarray(bounds, float)
    return System(name="he1d", bounds=b, n_g=n_g, centres=np.array([0.0]),
                  charges=np.array([2.0]), beta=beta, M=M)


def h3p_1d(R=1.8, half_width=60.0, n_e=60, n_g=6, beta=100.0, tau_kind="power",
           M=1024, u=64, p=16, bounds=None) -> System:
    """Linear 1D H3+: unit charges at -R, 0, +R (Sec. 3.2, Eq. h3pv).

    The paper prints the potential with its attraction sign lost and an offset
    5/d inside v; here v is attractive and the bare proton-proton repulsion
    1/R + 1/R + 1/(2R) = 5/(2R) is added once to the total energy.
    """
    b = uniform_bounds(half_width, n_e) if bounds is None else np.asarray(bounds, float)
    return System(name="h3p1d", bounds=b, n_g=n_g, centres=np.array([-R, 0.0, R]),
                  charges=np.array([1.0, 1.0, 1.0]), beta=beta, tau_kind=tau_kind,
                  M=M, u=u, p=p, e_nn=5.0 / (2.0 * R))


def harmonic_trap(n_elec=20.0, omega=1.0, half_width=12.0, n_e=101, n_g=5, beta=20.0, M=256,
                  ee_scale=0.5) -> System:
    """n_elec fermions (closed shells, both spins) in the trap (1/2) omega^2 x^2 with
    the soft-Coulomb interaction of Sec. 3 scaled by ee_scale; no nuclei. The
    default grid has n_b = 504 (101 equal elements x 6 GLL points on [-12, 12]),
    the size class the paper's conclusion names (N <= 20, n_b > 500)."""
    return System(name="trap1d", bounds=uniform_bounds(half_width, n_e), n_g=n_g, centres=np.zeros(0),
                  charges=np.zeros(0), ee_scale=ee_scale, n_elec=n_elec, beta=beta, M=M, omega=omega)


def config_he() -> System:
    """He, box [-10, 10], 4 elements x 6 GLL points (n_b = 19), beta = 50, 129 tau points."""
    return he_1d()


def config_sigma_bench() -> System:
    """Sigma-2B microbenchmark grid: [-40, 40], 40 elements x 6 GLL points (n_b = 199),
    beta = 50, 1025 tau points."""
    return he_1d(half_width=40.0, n_e=40, n_g=5, beta=50.0, M=1024)


def config_h3p() -> System:
    """H3+, R = 1.8, box [-60, 60], 60 elements x 7 GLL points (n_b = 359), beta = 100,
    power mesh u = 64, p = 16 (2049 tau points)."""
    return h3p_1d()


def scan_R(k: int, n: int = 64) -> float:
    return 1.0 + 2.0 * k / (n - 1)


def config_scan(n: int = 64, M: int = 1024) -> List[System]:
    """Bond-length scan of linear H3+: R uniform in [1, 3], box half-width 30 + 10 R,
    round(30 + 25 (R - 1)) equal elements of 6 GLL points, beta = 100, uniform tau grid."""
    out = []
    for k in range(n):
        R = scan_R(k, n)
        n_e = int(round(30 + 25 * (R - 1.0)))
        out.append(h3p_1d(R=R, half_width=30.0 + 10.0 * R, n_e=n_e, n_g=5, beta=100.0,
                          tau_kind="uniform", M=M))
    return out


def config_scan_small(n: int = 64, M: int = 1024) -> List[System]:
    """The same bond-length scan in short boxes: R uniform in [1, 3], box half-width
    10 + 2 R, round(6 + 4 (R - 1)) equal elements of 6 GLL points (n_b 29..69),
    beta = 100, uniform tau grid. Many small systems, none of which fills the GPU
    alone: the case in which batching them matters."""
    out = []
    for k in range(n):
        R = scan_R(k, n)
        n_e = int(round(6 + 4 * (R - 1.0)))
        out.append(h3p_1d(R=R, half_width=10.0 + 2.0 * R, n_e=n_e, n_g=5, beta=100.0,
                          tau_kind="uniform", M=M))
    return out


def random_potential_system(seed: int, base: System | None = None) -> System:
    """Two electrons in a seeded random soft-Coulomb potential: 1-3 centres,
    charges in [1, 2], positions in [-3, 3]; grid and tau grid of ``base``
    (default: the n_b = 199, beta = 50, 1025-point microbenchmark grid)."""
    base = config_sigma_bench() if base is None else base
    rng = np.random.default_rng(seed)
    n_c = int(rng.integers(1, 4))
    Z = rng.uniform(1.0, 2.0, size=n_c)
    X = rng.uniform(-3.0, 3.0, size=n_c)
    return base.with_(name=f"rand{seed}", centres=X, charges=Z)


# ---------------------------------------------------------------- seeded arrays

def synthetic_G(n_b: int, M: int, beta: float, seed: int = 2, dtype=np.float64) -> np.ndarray:
    """Seeded symmetric G(tau) on a uniform grid of M + 1 points.

    Each slice q is S_q * exp(-tau_q), tau_q = q beta / M, where S_q is exactly
    symmetric with every entry ~ N(0, 0.1^2): the upper triangle (with diagonal)
    of a Gaussian matrix mirrored into the lower triangle.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((M + 1, n_b, n_b), dtype=np.float64)
    iu = np.triu_indices(n_b)
    for q in range(M + 1):
        R = rng.normal(0.0, 0.1, size=(n_b, n_b))
        S = np.zeros((n_b, n_b))
        S[iu] = R[iu]
        S = S + np.triu(S, 1).T
        out[q] = S * np.exp(-q * beta / M)
    return out.astype(dtype, copy=False)


def random_symmetric_slices(n_b: int, n_tau: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """Seeded exactly-symmetric [n_tau][n_b][n_b] array, entries ~ N(0, scale^2)."""
    rng = np.random.default_rng(seed)
    A = rng.normal(0.0, scale, size=(n_tau, n_b, n_b))
    iu = np.triu_indices(n_b, 1)
    for q in range(n_tau):
        A[q][(iu[1], iu[0])] = A[q][iu]
    return A


def random_symmetric(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    return random_symmetric_slices(n, 1, seed, scale)[0]


def mlp_init(n_params_layers, seed: int = 0) -> np.ndarray:
    """Seeded initial parameters for a dense network given as [(fan_in, fan_out), ...]:
    weights uniform in +-sqrt(6 / (fan_in + fan_out)), biases zero, flattened layer by
    layer (weights row-major, then biases)."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in n_params_layers:
        lim = np.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts)
