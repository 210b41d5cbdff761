"""Imaginary-time convolutions, the Dyson step and the total energy
(paper Sec. 2.3, Eq. deq and the text after it).

Oracle (test infrastructure only). Plain float64.

Dyson equation on [0, beta] (Eq. deq, moved to tau > 0):
    G = G0 + I2,  I2(tau) = int_0^beta G0(tau - s) I1(s) ds,
    I1(tau) = (Sigma^HF[G] - Sigma0) G(tau) + int_0^beta Sigma_c(tau - s) G(s) ds,
with the antiperiodic continuation A(s - beta) = -A(s) for arguments in (-beta, 0).

Quadrature (the paper says only that the integrals are done "by direct
integration"; the rule below is this oracle's reading): the integral is
split at s = tau_p, and each part uses the trapezoid rule on the grid
points it covers, with the one-sided limits at the split point,

  Q_p[A, B] = sum_{q<=p} wL_pq A(tau_p - tau_q) B_q  -  sum_{q>=p} wR_pq A(beta + tau_p - tau_q) B_q,

A(0) meaning A(0^+) and A(beta) meaning A(beta^-). On a uniform grid the
kernel values are grid values. On the power mesh G0 is evaluated exactly and
Sigma_c between grid points by 4-point Lagrange interpolation inside the
uniform block that contains the argument.

Total energy (the paper computes it "similar as" in its cited works; the
Galitskii-Migdal form used here):
  E = sigma (Tr[h rho] + 1/2 Tr[Sigma^HF[rho] rho]) - (sigma/2) int Tr[Sigma_c(beta - tau) G(tau)] dtau,
rho = -G(beta^-), the tau integral by the plain trapezoid rule on the grid.
"""
from __future__ import annotations

import numpy as np

from .fedvr import trapezoid_weights
from .hf import sigma_hf, g0_diag, hf_energy


# ----------------------------------------------------------------------------- weights
def split_weights(t: np.ndarray, p: int):
    """Trapezoid weights on [t_0, t_p] (wL) and on [t_p, t_M] (wR), both of length M + 1."""
    n = len(t)
    wL = np.zeros(n)
    wR = np.zeros(n)
    if p > 0:
        wL[: p + 1] = trapezoid_weights(t[: p + 1])
    if p < n - 1:
        wR[p:] = trapezoid_weights(t[p:])
    return wL, wR


# ----------------------------------------------------------------------------- kernels
def lagrange4(t: np.ndarray, s: float, block: int):
    """Nodes and weights of 4-point Lagrange interpolation at s, with the stencil kept
    inside the uniform block [k block, (k+1) block] of node indices holding s."""
    n = len(t)
    a = int(np.searchsorted(t, s, side="right")) - 1
    a = min(max(a, 0), n - 2)
    lo = (a // block) * block
    hi = min(lo + block, n - 1)
    start = min(max(a - 1, lo), hi - 3)
    nodes = np.arange(start, start + 4)
    w = np.ones(4)
    for m in range(4):
        for j in range(4):
            if j != m:
                w[m] *= (s - t[nodes[j]]) / (t[nodes[m]] - t[nodes[j]])
    return nodes, w


def kernel_grid(A: np.ndarray, p: int, q: int, side: str):
    """Grid kernel on a uniform mesh: A(tau_p - tau_q) = A_{p-q} (side 'L', q <= p) and
    A(beta + tau_p - tau_q) = A_{M+p-q} (side 'R', q >= p)."""
    M = A.shape[0] - 1
    return A[p - q] if side == "L" else A[M + p - q]


def make_kernel_interp(A: np.ndarray, t: np.ndarray, block: int):
    beta = t[-1]

    def k(p, q, side):
        s = t[p] - t[q] if side == "L" else beta + t[p] - t[q]
        if side == "L" and p == q:
            return A[0]
        if side == "R" and p == q:
            return A[-1]
        nodes, w = lagrange4(t, s, block)
        return np.tensordot(w, A[nodes], axes=(0, 0))
    return k


def make_kernel_g0(hf, t: np.ndarray):
    """Exact G0 kernel: G0(s) = -C diag((1-f) e^(-s xi)) C^T at s = tau_p - tau_q (or
    beta + tau_p - tau_q), with s = 0 read as 0^+ and s = beta as beta^-."""
    beta = t[-1]

    def k(p, q, side):
        if side == "L":
            s = 0.0 if p == q else t[p] - t[q]
        else:
            s = beta if p == q else beta + t[p] - t[q]
        g = g0_diag(hf.eps - hf.mu, np.array([s]), hf.beta)[0]
        return -(hf.C * g) @ hf.C.T
    return k


# ----------------------------------------------------------------------------- Q
def conv_direct(kernel, B: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Q_p[A, B] for every p by the literal split-trapezoid double sum."""
    n_t = B.shape[0]
    out = np.zeros_like(B)
    for p in range(n_t):
        wL, wR = split_weights(t, p)
        acc = np.zeros_like(B[0])
        for q in range(p + 1):
            if wL[q] != 0.0:
                acc += wL[q] * (kernel(p, q, "L") @ B[q])
        for q in range(p, n_t):
            if wR[q] != 0.0:
                acc -= wR[q] * (kernel(p, q, "R") @ B[q])
        out[p] = acc
    return out


def conv_uniform_fft(A: np.ndarray, B: np.ndarray, dtau: float) -> np.ndarray:
    """Q_p[A, B] on a uniform grid via the discrete Fourier transform.

    For 0 < p < M the split-trapezoid sum equals dtau * sum_{q<M} At_{p-q} Bh_q, an
    antiperiodic circular convolution of length M, where Ah_0 = (A_0 - A_M)/2,
    Bh_0 = (B_0 - B_M)/2 (jump averages) and At is the antiperiodic extension of Ah.
    Twisting by e^(-i pi q / M) makes it periodic (odd Matsubara frequencies).
    The end points differ from the circular sum only in the q = 0 / q = M terms,
    which are corrected explicitly; Q_M = -Q_0.
    """
    M = A.shape[0] - 1
    Ah = A[:M].copy()
    Ah[0] = 0.5 * (A[0] - A[M])
    Bh = B[:M].copy()
    Bh[0] = 0.5 * (B[0] - B[M])
    tw = np.exp(-1j * np.pi * np.arange(M) / M)[:, None, None]
    Af = np.fft.fft(Ah * tw, axis=0)
    Bf = np.fft.fft(Bh * tw, axis=0)
    c = (np.fft.ifft(Af @ Bf, axis=0) * np.conj(tw)).real
    Q = np.empty_like(B)
    Q[1:M] = dtau * c[1:M]
    Q0 = dtau * (c[0] - Ah[0] @ Bh[0] - 0.5 * (A[M] @ B[0]) - 0.5 * (A[0] @ B[M]))
    Q[0] = Q0
    Q[M] = -Q0
    return Q


# ----------------------------------------------------------------------------- step
class DysonContext:
    """What a Dyson step needs besides G and Sigma_c."""

    def __init__(self, setup, hf, tau_kind: str, block: int = 0):
        self.V, self.h = setup.V, setup.h
        self.sigma = setup.sys.sigma
        self.t = setup.tau
        self.hf = hf
        self.kind = tau_kind
        self.block = block
        from .hf import g0_tau
        self.G0 = g0_tau(hf, self.t)


def conv(ctx: DysonContext, which: str, A: np.ndarray, B: np.ndarray, route: str) -> np.ndarray:
    """Q[A, B] with A = Sigma_c (which='sigma') or A = G0 (which='g0')."""
    t = ctx.t
    if ctx.kind == "uniform":
        M = len(t) - 1
        if route == "fft":
            return conv_uniform_fft(A, B, t[-1] / M)
        return conv_direct(lambda p, q, s: kernel_grid(A, p, q, s), B, t)
    if which == "g0":
        return conv_direct(make_kernel_g0(ctx.hf, t), B, t)
    return conv_direct(make_kernel_interp(A, t, ctx.block), B, t)


def dyson_step(ctx: DysonContext, G: np.ndarray, Sc: np.ndarray, alpha: float,
               symmetrize: bool = True, route: str = "fft") -> np.ndarray:
    """One sequential solution of Eq. deq followed by linear mixing:

    rho = -G(beta^-); St = Sigma^HF[rho] - Sigma0; I1_p = St G_p + Q_p[Sigma_c, G];
    I2_p = Q_p[G0, I1]; G_new = G0 + I2; G <- (1 - alpha) G + alpha G_new; then
    G <- (G + G^T)/2 slice by slice when ``symmetrize``.
    """
    rho = -G[-1]
    St = sigma_hf(ctx.V, rho, ctx.sigma) - ctx.hf.Sigma0
    I1 = np.einsum("ik,qkj->qij", St, G) + conv(ctx, "sigma", Sc, G, route)
    I2 = conv(ctx, "g0", ctx.G0, I1, route)
    Gn = (1.0 - alpha) * G + alpha * (ctx.G0 + I2)
    if symmetrize:
        Gn = 0.5 * (Gn + Gn.transpose(0, 2, 1))
    return Gn


def gm_energy(h, V, sigma, G, Sc, t, e_nn=0.0):
    """Galitskii-Migdal total energy of G with its correlation self-energy Sc."""
    rho = -G[-1]
    E1 = hf_energy(h, V, rho, sigma)
    w = trapezoid_weights(t)
    tr = np.einsum("qij,qji->q", Sc[::-1], G)
    return E1 - 0.5 * sigma * float(np.sum(w * tr)) + e_nn


def particle_number(G, sigma):
    """N = -sigma Tr G(beta^-) (the paper's N = sum_i g_ii(0^-) per spin, times sigma)."""
    return -sigma * float(np.trace(G[-1]))
