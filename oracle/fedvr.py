"""FE-DVR grid, quadrature and one- and two-body matrices (paper Sec. 2.1-2.2).

Oracle (test infrastructure only). Plain float64.

Reading of the paper's notation used throughout: ``N`` = n_g = number of basis
functions per element = Legendre degree; each element carries N + 1
generalized Gauss-Lobatto (GLL) points (the endpoints and the N - 1 roots of
P_N'), and the global basis has n_b = n_e N - 1 functions (Eq. basisdim).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L


# ----------------------------------------------------------------------------- O1
def gll_points(N: int):
    """GLL points and weights on [-1, 1] (Sec. 2.1, the GGL point and weight equations).

    Points: -1, +1 and the roots of d/dx P_N. Weights: w_m = 2 / (N (N+1) P_N(x_m)^2).
    The interior roots come from numpy's Legendre-series root finder and are
    polished by Newton steps on P_N'.
    """
    if N < 1:
        raise ValueError("need N >= 1")
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    d1 = L.legder(cN)
    d2 = L.legder(d1)
    if N >= 2:
        r = np.sort(np.real(L.legroots(d1)))
        for _ in range(4):
            r = r - L.legval(r, d1) / L.legval(r, d2)
        x = np.concatenate(([-1.0], r, [1.0]))
    else:
        x = np.array([-1.0, 1.0])
    PN = L.legval(x, cN)
    w = 2.0 / (N * (N + 1) * PN ** 2)
    return x, w


def lagrange_derivative_matrix(x: np.ndarray) -> np.ndarray:
    """D[m, b] = d/dx of the Lagrange polynomial through the nodes x that is 1 at
    x_b and 0 at the other nodes, evaluated at x_m (the Lobatto shape functions of
    Sec. 2.1 on the reference element). Written out by the product rule."""
    n = len(x)
    D = np.zeros((n, n))
    for m in range(n):
        for b in range(n):
            s = 0.0
            for k in range(n):
                if k == b:
                    continue
                t = 1.0 / (x[b] - x[k])
                for l in range(n):
                    if l != b and l != k:
                        t *= (x[m] - x[l]) / (x[b] - x[l])
                s += t
            D[m, b] = s
    return D


# ----------------------------------------------------------------------------- O2-O3
class Grid:
    """Global FE-DVR basis on the elements [bounds[e], bounds[e+1]] (Sec. 2.1).

    Attributes
        x[a], W[a]   node and summed GLL weight of basis function a
        idx[e, m]    global index of local node m of element e, -1 for the two
                     outer boundary nodes dropped by the Dirichlet condition
        xe[e], we[e] element nodes and weights (Eqs. xim, wim)
    Bridge functions (shared node between elements e and e+1) get the weight
    w^e_N + w^(e+1)_0 (Eq. basis); basis functions are ordered left to right.
    """

    def __init__(self, bounds, N: int):
        bounds = np.asarray(bounds, dtype=np.float64)
        self.bounds = bounds
        self.N = N
        self.n_e = len(bounds) - 1
        self.n_b = self.n_e * N - 1
        self.xg, self.wg = gll_points(N)
        self.D = lagrange_derivative_matrix(self.xg)
        n_e, n_b = self.n_e, self.n_b
        self.idx = np.full((n_e, N + 1), -1, dtype=np.int64)
        self.x = np.zeros(n_b)
        self.W = np.zeros(n_b)
        self.xe = np.zeros((n_e, N + 1))
        self.we = np.zeros((n_e, N + 1))
        a = 0
        for e in range(n_e):
            lo, hi = bounds[e], bounds[e + 1]
            h = hi - lo
            self.xe[e] = 0.5 * (h * self.xg + (hi + lo))       # Eq. xim
            self.we[e] = 0.5 * self.wg * h                      # Eq. wim
            for m in range(N + 1):
                if m == 0:
                    if e == 0:
                        continue                                # left Dirichlet end
                    g = self.idx[e - 1, N]                      # bridge with element e-1
                    self.idx[e, 0] = g
                    self.W[g] += self.we[e, 0]
                    continue
                if m == N and e == n_e - 1:
                    continue                                    # right Dirichlet end
                self.idx[e, m] = a
                self.x[a] = self.xe[e, m]
                self.W[a] += self.we[e, m]
                a += 1
        assert a == n_b


# ----------------------------------------------------------------------------- O4
def kinetic(grid: Grid) -> np.ndarray:
    """Kinetic matrix T_ab = (1/2) int chi_a' chi_b' dx (Sec. 2.2, Eq. tmat).

    Per element, t~_ab = sum_m f_a'(x_m) f_b'(x_m) w_m with the element's GLL rule
    (exact for the degree 2N-2 integrand); f' = (2/h) D on the reference element,
    so t~ = (2/h) sum_m w_m D_ma D_mb. Each basis function is f/sqrt(W) on every
    element it touches, which assembles the four cases of Eq. tmat.
    """
    n_b = grid.n_b
    T = np.zeros((n_b, n_b))
    N = grid.N
    for e in range(grid.n_e):
        h = grid.bounds[e + 1] - grid.bounds[e]
        te = (2.0 / h) * (grid.D.T @ (grid.wg[:, None] * grid.D))
        for a in range(N + 1):
            ga = grid.idx[e, a]
            if ga < 0:
                continue
            for b in range(N + 1):
                gb = grid.idx[e, b]
                if gb < 0:
                    continue
                T[ga, gb] += 0.5 * te[a, b] / np.sqrt(grid.W[ga] * grid.W[gb])
    return T


# ----------------------------------------------------------------------------- O5
def soft_coulomb_potential(x, centres, charges, soft=1.0) -> np.ndarray:
    """v(x) = -sum_c Z_c / sqrt((x - X_c)^2 + soft) (Sec. 3.1 helium, Sec. 3.2 H3+).
    In the DVR the potential matrix is diagonal with entries v(x_a) (Eq. vmat)."""
    x = np.asarray(x, dtype=np.float64)
    v = np.zeros_like(x)
    for X, Z in zip(centres, charges):
        v -= Z / np.sqrt((x - X) ** 2 + soft)
    return v


def harmonic_potential(x, omega) -> np.ndarray:
    """Harmonic confinement (1/2) omega^2 x^2 (the trap of the paper's conclusion),
    diagonal in the DVR like any local potential (Eq. vmat)."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * omega * omega * x * x


# ----------------------------------------------------------------------------- O6
def interaction_direct(x, ee_soft=1.0, scale=1.0) -> np.ndarray:
    """Diagonal-pair interaction kernel V_ab = u(|x_a - x_b|), u = scale / sqrt(d^2 + ee_soft)
    (Sec. 2.2, Eqs. umat1, umatred; Sec. 3 for u)."""
    d = x[:, None] - x[None, :]
    return scale / np.sqrt(d * d + ee_soft)


def interaction_eigen_route(grid: Grid, ee_soft=1.0, scale=1.0) -> np.ndarray:
    """The paper's route to the kernel (Eqs. umatred, umatsep): diagonalise
    U_(em),(e'm') = u(|x^e_m - x^e'_m'|) over all element-local nodes (bridge
    points appear twice, the two Dirichlet end points are left out), form
    beta from the eigenvectors with the weighted average on bridges, and sum
    alpha beta beta. Kept to pin that it equals interaction_direct."""
    loc = []
    for e in range(grid.n_e):
        for m in range(grid.N + 1):
            if grid.idx[e, m] >= 0:
                loc.append((e, m))
    xl = np.array([grid.xe[e, m] for e, m in loc])
    d = xl[:, None] - xl[None, :]
    U = scale / np.sqrt(d * d + ee_soft)
    alpha, bt = np.linalg.eigh(U)
    pos = {em: r for r, em in enumerate(loc)}
    n_b = grid.n_b
    beta = np.zeros((n_b, len(loc)))
    N = grid.N
    for e in range(grid.n_e):
        for m in range(1, N + 1):
            g = grid.idx[e, m]
            if g < 0:
                continue
            if m == N and e + 1 < grid.n_e:
                # bridge: weighted average of the two copies (Eq. for beta, m = 0 case)
                w1, w2 = grid.we[e, N], grid.we[e + 1, 0]
                beta[g] = (bt[pos[(e, N)]] * w1 + bt[pos[(e + 1, 0)]] * w2) / (w1 + w2)
            else:
                beta[g] = bt[pos[(e, m)]]
    return (beta * alpha[None, :]) @ beta.T


# ----------------------------------------------------------------------------- tau grids
def tau_uniform(beta: float, M: int) -> np.ndarray:
    """M + 1 equidistant points on [0, beta]; the second half is the mirror
    image beta - tau of the first, so the grid is exactly symmetric."""
    t = np.zeros(M + 1)
    for q in range(M // 2 + 1):
        t[q] = beta * q / M
    for q in range(M // 2 + 1, M + 1):
        t[q] = beta - t[M - q]
    return t


def tau_power(beta: float, u: int, p: int) -> np.ndarray:
    """Power mesh with 2 u p + 1 points (Sec. 3.1: the mesh of the cited power-mesh
    method). Reading: breakpoints 0, beta/2^p, beta/2^(p-1), ..., beta/2; each of the
    p intervals is split into u equal steps; the second half mirrors the first."""
    half = [0.0]
    brk = [0.0] + [beta / 2.0 ** (p - k) for k in range(p)]      # 0, b/2^p, ..., b/2
    for k in range(p):
        a, b = brk[k], brk[k + 1]
        for j in range(1, u + 1):
            half.append(a + (b - a) * j / u)
    half = np.array(half)                                         # u p + 1 points, ends at beta/2
    half[-1] = beta / 2.0
    n = 2 * u * p + 1
    t = np.zeros(n)
    t[: u * p + 1] = half
    for q in range(u * p + 1, n):
        t[q] = beta - t[n - 1 - q]
    return t


def trapezoid_weights(t: np.ndarray) -> np.ndarray:
    """Plain trapezoid weights on the points t (end values included)."""
    w = np.zeros_like(t)
    dt = np.diff(t)
    w[:-1] += 0.5 * dt
    w[1:] += 0.5 * dt
    return w


# ----------------------------------------------------------------------------- bundle
class Setup:
    """Everything the Dyson iteration needs from the grid: x, W, T, v, V, h = T + diag(v)."""

    def __init__(self, sysd):
        self.sys = sysd
        self.grid = Grid(sysd.bounds, sysd.n_g)
        self.x = self.grid.x
        self.W = self.grid.W
        self.T = kinetic(self.grid)
        self.v = soft_coulomb_potential(self.x, sysd.centres, sysd.charges, sysd.soft)
        if getattr(sysd, "omega", 0.0):
            self.v = self.v + harmonic_potential(self.x, sysd.omega)
        self.V = interaction_direct(self.x, sysd.ee_soft, sysd.ee_scale)
        self.h = self.T + np.diag(self.v)
        if sysd.tau_kind == "uniform":
            self.tau = tau_uniform(sysd.beta, sysd.M)
        elif sysd.tau_kind == "power":
            self.tau = tau_power(sysd.beta, sysd.u, sysd.p)
        else:
            raise ValueError(sysd.tau_kind)
