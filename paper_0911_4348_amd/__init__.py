"""Python binding of the MI355X FE-DVR second-Born library (``libnegf.so``).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels (or, for the FE-DVR setup and tau grids, its host C++).
PyTorch is used for device memory and streams. The C names and their
documentation are in ``include/negf.h``.

If the shared library has not been built, importing this module still works
but every call raises ``RuntimeError``; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnegf.so")

OK, EINVAL, ENODEV, EHIP, ENAN, ENOCONV, ENOMEM = 0, -1, -2, -3, -4, -5, -6
F64, F32, BF16 = 0, 1, 2
TAU_UNIFORM, TAU_POWER = 0, 1
CONV_AUTO, CONV_FFT, CONV_DIRECT = 0, 1, 2
STOP_DELTA, STOP_CONTRACTION = 0, 1
_STOP = {"delta": STOP_DELTA, "contraction": STOP_CONTRACTION, STOP_DELTA: STOP_DELTA,
         STOP_CONTRACTION: STOP_CONTRACTION}
N_CFG = 13              # Sigma-2B tile configurations (negf_sigma2b_set_config)

_NAMES = {OK: "NEGF_OK", EINVAL: "NEGF_EINVAL", ENODEV: "NEGF_ENODEV", EHIP: "NEGF_EHIP",
          ENAN: "NEGF_ENAN", ENOCONV: "NEGF_ENOCONV", ENOMEM: "NEGF_ENOMEM"}


class NegfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


# ------------------------------------------------------------------ C structs
class GridT(C.Structure):
    _fields_ = [("n_e", C.c_int), ("n_g", C.c_int), ("bounds", C.POINTER(C.c_double))]


class PotentialT(C.Structure):
    _fields_ = [("n_c", C.c_int), ("X", C.POINTER(C.c_double)), ("Z", C.POINTER(C.c_double)),
                ("soft", C.c_double), ("ee_soft", C.c_double), ("ee_scale", C.c_double), ("omega", C.c_double)]


class TauGridT(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_tau", C.c_int), ("block", C.c_int), ("beta", C.c_double),
                ("tau", C.POINTER(C.c_double))]


class SystemT(C.Structure):
    _fields_ = [("grid", GridT), ("pot", PotentialT), ("n_elec", C.c_double), ("sigma", C.c_int),
                ("beta", C.c_double), ("tau_kind", C.c_int), ("M", C.c_int), ("u", C.c_int),
                ("p", C.c_int), ("e_nn", C.c_double)]


class OptsT(C.Structure):
    _fields_ = [("alpha", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int),
                ("fixed_iters", C.c_int), ("dtype", C.c_int), ("conv_algo", C.c_int),
                ("symmetrize", C.c_int), ("refine_tol", C.c_double), ("hf_tol", C.c_double),
                ("hf_max_iter", C.c_int), ("guess_params", C.c_void_p), ("guess_scale", C.c_double),
                ("tune", C.c_int), ("no_graph", C.c_int), ("progress", C.c_int), ("stop_rule", C.c_int),
                ("guard", C.c_int)]


class IterLogT(C.Structure):
    _fields_ = [("iter", C.c_int), ("dtype", C.c_int), ("E", C.c_double), ("dE", C.c_double),
                ("N", C.c_double), ("ms", C.c_double)]


# ------------------------------------------------------------------ loading
_lib = None

_VP, _DP, _IP = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
_SIGS = {
    "negf_last_error": (C.c_char_p, []),
    "negf_version": (C.c_int, []),
    "negf_ctx_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    "negf_ctx_destroy": (C.c_int, [_VP]),
    "negf_ctx_scratch_bytes": (C.c_int, [_VP, C.POINTER(C.c_size_t)]),
    "negf_fedvr_size": (C.c_int, [C.c_int, C.c_int, _IP]),
    "fedvr_build": (C.c_int, [C.POINTER(GridT), C.POINTER(PotentialT), _DP, _DP, _DP, _DP, _DP]),
    "negf_density": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int, _VP, _VP, C.c_int, _VP, _VP]),
    "negf_density_at": (C.c_int, [C.POINTER(GridT), _DP, C.c_int, C.c_int, _DP, _DP]),
    "negf_tau_count": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, _IP]),
    "negf_tau_grid": (C.c_int, [C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, _DP]),
    "negf_hf": (C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_double, C.c_int, C.c_double, C.c_double,
                          C.c_int, _VP, _VP, _VP, _VP, _DP, _DP, _IP, _VP]),
    "negf_hf_batched": (C.c_int, [_VP, C.c_int, C.c_int, _VP, _VP, _VP, C.c_double, C.c_int, C.c_double, C.c_double,
                          C.c_int, _VP, _VP, _VP, _VP, _DP, _DP, _IP, _VP]),
    "negf_g0_build": (C.c_int, [_VP, C.c_int, C.c_int, _DP, C.c_double, _VP, _VP, C.c_double, _VP,
                                C.c_int, _VP]),
    "negf_sigma2b": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int, _VP, _VP, _VP, C.c_int, _VP]),
    "negf_sigma2b_noalloc": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int, _VP, _VP, _VP, C.c_int, _VP]),
    "negf_sigma2b_tune": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int, _VP, _VP, _VP, C.c_int, _IP, _DP, _VP]),
    "negf_sigma2b_set_config": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int]),
    "negf_dyson_step": (C.c_int, [_VP, C.POINTER(TauGridT), C.c_int, C.c_int, _VP, _VP, _VP, _VP,
                                  C.c_double, _VP, _VP, _VP, C.c_double, C.c_int, C.c_int, C.c_int,
                                  _VP, _DP, _DP, _VP]),
    "negf_energy": (C.c_int, [_VP, C.POINTER(TauGridT), C.c_int, C.c_int, _VP, _VP, _VP, _VP, C.c_int,
                              _DP, _DP, _VP]),
    "negf_scf": (C.c_int, [_VP, C.POINTER(SystemT), C.POINTER(OptsT), _VP, _VP, _DP, _DP, _IP,
                           C.POINTER(IterLogT), C.c_int, _DP, _DP, _VP]),
    "negf_scf_batched": (C.c_int, [_VP, C.c_int, C.POINTER(SystemT), C.POINTER(OptsT), _VP, _VP, _DP, _DP, _IP,
                                   _IP, C.POINTER(IterLogT), C.c_int, _IP, _DP, _DP, _VP]),
    "negf_sigma2b_batched": (C.c_int, [_VP, C.c_int, _IP, C.c_int, _IP, _VP, _VP, _VP, C.c_int, _VP]),
    "negf_sigma2b_batched_set_config": (C.c_int, [_VP, C.c_int, _IP, C.c_int, C.c_int]),
    "negf_sigma2b_batched_tune": (C.c_int, [_VP, C.c_int, _IP, C.c_int, _IP, _VP, _VP, _VP, C.c_int, C.c_int,
                                            _IP, _DP, _VP]),
    "negf_matrix_rate": (C.c_int, [_VP, C.c_int, _DP, _DP, _VP]),
    "negf_f64_issue_probe": (C.c_int, [_VP, C.c_int, C.c_int, _DP, _DP, _DP, _VP]),
    "negf_mlp_param_count": (C.c_int, [_IP]),
    "negf_mlp_features": (C.c_int, [_VP, C.c_int, _VP, _VP, C.c_int, _DP, _DP, C.c_int, _VP, C.c_double,
                                    C.c_int, _VP, _VP, _VP, _VP, _VP]),
    "negf_mlp_targets": (C.c_int, [_VP, C.c_int, _VP, _VP, C.c_double, _VP, C.c_int, _DP, C.c_int, _VP, C.c_double,
                                   C.c_int, _VP, _VP, _VP, _VP, _VP]),
    "negf_mlp_envelope": (C.c_int, [_VP, _VP, C.c_int, _DP, _VP, C.c_double, C.c_int, _VP, _VP, _VP, _VP, _VP]),
    "negf_mlp_forward": (C.c_int, [_VP, _VP, C.c_int, _VP, _VP, _VP]),
    "negf_mlp_train_step": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int, C.c_double, C.c_int, _VP, _VP, _VP, _DP,
                                      _VP]),
    "negf_mlp_guess": (C.c_int, [_VP, _VP, C.c_double, C.c_int, _VP, _VP, C.c_int, _DP, _DP, C.c_int, _VP,
                                 C.c_double, _VP, _VP, C.c_int, _VP]),
}


def lib():
    """The loaded shared library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_0911_4348_amd/build.py "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise NegfError(rc, lib().negf_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


# ------------------------------------------------------------------ torch helpers
def _torch():
    import torch
    return torch


def _dev_ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


_DT = {"f64": F64, "f32": F32, "bf16": BF16, F64: F64, F32: F32, BF16: BF16}


def _tensor_dtype(dt):
    torch = _torch()
    return torch.float64 if _DT[dt] == F64 else torch.float32


# ------------------------------------------------------------------ context
class Context:
    """A library context on one GPU (owns the device scratch)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().negf_ctx_create(device, C.byref(h)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def scratch_bytes(self) -> int:
        b = C.c_size_t()
        _check(lib().negf_ctx_scratch_bytes(self._h, C.byref(b)))
        return b.value

    def close(self):
        if getattr(self, "_h", None):
            lib().negf_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ setup (host)
def fedvr_size(n_e: int, n_g: int) -> int:
    n = C.c_int()
    _check(lib().negf_fedvr_size(n_e, n_g, C.byref(n)))
    return n.value


def _grid_pot(bounds, n_g, centres, charges, soft, ee_soft, ee_scale, omega=0.0):
    b = np.ascontiguousarray(bounds, dtype=np.float64)
    X = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1)
    Z = np.ascontiguousarray(charges, dtype=np.float64).reshape(-1)
    g = GridT(len(b) - 1, n_g, _dptr(b))
    p = PotentialT(len(X), _dptr(X) if len(X) else None, _dptr(Z) if len(Z) else None,
                   soft, ee_soft, ee_scale, omega)
    return g, p, (b, X, Z)


def fedvr_build(bounds, n_g, centres, charges, soft=1.0, ee_soft=1.0, ee_scale=1.0, omega=0.0):
    """Host FE-DVR setup; returns numpy (x, W, T, v, V)."""
    g, p, keep = _grid_pot(bounds, n_g, centres, charges, soft, ee_soft, ee_scale, omega)
    n = fedvr_size(g.n_e, n_g)
    x, W, v = np.zeros(n), np.zeros(n), np.zeros(n)
    T, V = np.zeros((n, n)), np.zeros((n, n))
    _check(lib().fedvr_build(C.byref(g), C.byref(p), _dptr(x), _dptr(W), _dptr(T), _dptr(v), _dptr(V)))
    return x, W, T, v, V


def fedvr_build_system(sysd):
    return fedvr_build(sysd.bounds, sysd.n_g, sysd.centres, sysd.charges, sysd.soft, sysd.ee_soft,
                       sysd.ee_scale, getattr(sysd, "omega", 0.0))


def density_at(bounds, n_g, rho, sigma, xs) -> np.ndarray:
    """negf_density_at: n(x) at the points xs from the per-spin density matrix rho (host)."""
    b = np.ascontiguousarray(bounds, dtype=np.float64)
    r = np.ascontiguousarray(rho, dtype=np.float64)
    x = np.ascontiguousarray(xs, dtype=np.float64)
    out = np.zeros(len(x))
    g = GridT(len(b) - 1, n_g, _dptr(b))
    _check(lib().negf_density_at(C.byref(g), _dptr(r), int(sigma), len(x), _dptr(x), _dptr(out)))
    return out


def tau_grid(kind, beta, M=0, u=0, p=0) -> np.ndarray:
    kind = TAU_UNIFORM if kind in ("uniform", TAU_UNIFORM) else TAU_POWER
    n = C.c_int()
    _check(lib().negf_tau_count(kind, M, u, p, C.byref(n)))
    t = np.zeros(n.value)
    _check(lib().negf_tau_grid(kind, beta, M, u, p, _dptr(t)))
    return t


def tau_grid_system(sysd) -> np.ndarray:
    return tau_grid(sysd.tau_kind, sysd.beta, sysd.M, sysd.u, sysd.p)


class TauGrid:
    """Host description of a tau grid, kept alive for the C struct."""

    def __init__(self, kind, beta, tau: np.ndarray, block: int = 0):
        self.kind = TAU_UNIFORM if kind in ("uniform", TAU_UNIFORM) else TAU_POWER
        self.beta = float(beta)
        self.tau = np.ascontiguousarray(tau, dtype=np.float64)
        self.block = int(block)
        self.struct = TauGridT(self.kind, len(self.tau), self.block, self.beta, _dptr(self.tau))

    @classmethod
    def of_system(cls, sysd):
        return cls(sysd.tau_kind, sysd.beta, tau_grid_system(sysd),
                   sysd.u if sysd.tau_kind == "power" else 0)


# ------------------------------------------------------------------ device calls
@dataclass
class HFState:
    eps: object
    C: object
    rho: object
    Sigma0: object
    mu: float
    E: float
    iters: int


def hf(ctx: Context, T, v, V, n_elec, sigma, beta, tol=1e-13, max_iter=1000, stream=None) -> HFState:
    """negf_hf on device tensors T, v, V (float64)."""
    torch = _torch()
    n = v.shape[0]
    dev = T.device
    eps = torch.empty(n, dtype=torch.float64, device=dev)
    Cm = torch.empty((n, n), dtype=torch.float64, device=dev)
    rho = torch.empty((n, n), dtype=torch.float64, device=dev)
    S0 = torch.empty((n, n), dtype=torch.float64, device=dev)
    mu, E, it = C.c_double(), C.c_double(), C.c_int()
    _check(lib().negf_hf(ctx.handle, n, _dev_ptr(T), _dev_ptr(v), _dev_ptr(V), float(n_elec), int(sigma),
                         float(beta), float(tol), int(max_iter), _dev_ptr(eps), _dev_ptr(Cm), _dev_ptr(rho),
                         _dev_ptr(S0), C.byref(mu), C.byref(E), C.byref(it), _stream(stream)))
    return HFState(eps, Cm, rho, S0, mu.value, E.value, it.value)


def hf_batched(ctx: Context, T, v, V, n_elec, sigma, beta, tol=1e-13, max_iter=1000, allow_noconv=False,
               stream=None):
    """negf_hf_batched on stacked device tensors T[B,n,n], v[B,n], V[B,n,n] (float64).
    Returns (eps[B,n], C[B,n,n], rho[B,n,n], Sigma0[B,n,n], mu[B], E_hf[B], iters[B]); the last
    three are numpy arrays."""
    torch = _torch()
    B, n = v.shape
    dev = T.device
    eps = torch.empty((B, n), dtype=torch.float64, device=dev)
    Cm = torch.empty((B, n, n), dtype=torch.float64, device=dev)
    rho = torch.empty((B, n, n), dtype=torch.float64, device=dev)
    S0 = torch.empty((B, n, n), dtype=torch.float64, device=dev)
    mu = np.zeros(B)
    E = np.zeros(B)
    it = np.zeros(B, dtype=np.int32)
    rc = (lib().negf_hf_batched(ctx.handle, B, n, _dev_ptr(T), _dev_ptr(v), _dev_ptr(V), float(n_elec),
                                 int(sigma), float(beta), float(tol), int(max_iter), _dev_ptr(eps), _dev_ptr(Cm),
                                 _dev_ptr(rho), _dev_ptr(S0), _dptr(mu), _dptr(E),
                                 it.ctypes.data_as(_IP), _stream(stream)))
    if rc != OK and not (allow_noconv and rc == ENOCONV):
        _check(rc)
    return eps, Cm, rho, S0, mu, E, it


def g0_build(ctx: Context, hfs: HFState, tau: np.ndarray, beta, dtype="f64", stream=None):
    torch = _torch()
    n = hfs.eps.shape[0]
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    G0 = torch.empty((len(tau), n, n), dtype=_tensor_dtype(dtype), device=hfs.eps.device)
    _check(lib().negf_g0_build(ctx.handle, n, len(tau), _dptr(tau), float(beta), _dev_ptr(hfs.eps),
                               _dev_ptr(hfs.C), float(hfs.mu), _dev_ptr(G0), _DT[dtype], _stream(stream)))
    return G0


def sigma2b(ctx: Context, V, G, sigma: int, dtype="f64", out=None, stream=None):
    """negf_sigma2b: returns Sigma_c with the shape of G."""
    torch = _torch()
    n_tau, n, _ = G.shape
    if out is None:
        out = torch.empty_like(G)
    _check(lib().negf_sigma2b(ctx.handle, n, n_tau, int(sigma), _dev_ptr(V), _dev_ptr(G), _dev_ptr(out),
                              _DT[dtype], _stream(stream)))
    return out


def sigma2b_noalloc(ctx: Context, V, G, sigma: int, out, dtype="f64", stream=None):
    """negf_sigma2b_noalloc: Sigma_c into the caller's ``out`` (same shape as G);
    float64 or float32 only, no allocation by the library or by this wrapper."""
    n_tau, n, _ = G.shape
    _check(lib().negf_sigma2b_noalloc(ctx.handle, n, n_tau, int(sigma), _dev_ptr(V), _dev_ptr(G), _dev_ptr(out),
                                      _DT[dtype], _stream(stream)))
    return out


def sigma2b_tune(ctx: Context, V, G, sigma: int, dtype="f64", out=None, stream=None):
    """negf_sigma2b_tune: returns (best config index, per-config milliseconds)."""
    torch = _torch()
    n_tau, n, _ = G.shape
    if out is None:
        out = torch.empty_like(G)
    best = C.c_int()
    ms = (C.c_double * N_CFG)()
    _check(lib().negf_sigma2b_tune(ctx.handle, n, n_tau, int(sigma), _dev_ptr(V), _dev_ptr(G), _dev_ptr(out),
                                   _DT[dtype], C.byref(best), ms, _stream(stream)))
    return best.value, list(ms)


def sigma2b_set_config(ctx: Context, n_b: int, dtype: str, cfg: int):
    _check(lib().negf_sigma2b_set_config(ctx.handle, int(n_b), _DT[dtype], int(cfg)))


def dyson_step(ctx: Context, tg: TauGrid, sigma, h, V, hfs: HFState, G_in, Sc, alpha, symmetrize=True,
               conv=CONV_AUTO, dtype="f64", G_out=None, want_energy=True, stream=None):
    """negf_dyson_step; returns (G_out, E, N) (E, N of G_in, None if not requested)."""
    torch = _torch()
    n = G_in.shape[1]
    if G_out is None:
        G_out = torch.empty_like(G_in)
    E, N = C.c_double(), C.c_double()
    _check(lib().negf_dyson_step(ctx.handle, C.byref(tg.struct), n, int(sigma), _dev_ptr(h), _dev_ptr(V),
                                 _dev_ptr(hfs.eps), _dev_ptr(hfs.C), float(hfs.mu), _dev_ptr(hfs.Sigma0),
                                 _dev_ptr(G_in), _dev_ptr(Sc), float(alpha), int(symmetrize), int(conv),
                                 _DT[dtype], _dev_ptr(G_out), C.byref(E) if want_energy else None,
                                 C.byref(N) if want_energy else None, _stream(stream)))
    return G_out, (E.value if want_energy else None), (N.value if want_energy else None)


def density(ctx: Context, W, G, sigma, dtype="f64", out=None, stream=None):
    """negf_density: n at the DVR nodes from G(beta^-); W, G device tensors."""
    torch = _torch()
    n_tau, n, _ = G.shape
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=G.device)
    _check(lib().negf_density(ctx.handle, n, n_tau, int(sigma), _dev_ptr(W), _dev_ptr(G), _DT[dtype], _dev_ptr(out),
                              _stream(stream)))
    return out


def energy(ctx: Context, tg: TauGrid, sigma, h, V, G, Sc, dtype="f64", stream=None):
    n = G.shape[1]
    E, N = C.c_double(), C.c_double()
    _check(lib().negf_energy(ctx.handle, C.byref(tg.struct), n, int(sigma), _dev_ptr(h), _dev_ptr(V),
                             _dev_ptr(G), _dev_ptr(Sc), _DT[dtype], C.byref(E), C.byref(N), _stream(stream)))
    return E.value, N.value


@dataclass
class SCFOut:
    G: object
    E: float
    N: float
    iters: int
    hf_E: float
    hf_mu: float
    log: list
    status: int


def system_struct(sysd):
    """Build the C negf_system_t for a workloads.System (returns struct, keep-alive)."""
    g, p, keep = _grid_pot(sysd.bounds, sysd.n_g, sysd.centres, sysd.charges, sysd.soft, sysd.ee_soft,
                           sysd.ee_scale, getattr(sysd, "omega", 0.0))
    kind = TAU_UNIFORM if sysd.tau_kind == "uniform" else TAU_POWER
    s = SystemT(g, p, float(sysd.n_elec), int(sysd.sigma), float(sysd.beta), kind, int(sysd.M),
                int(sysd.u), int(sysd.p), float(sysd.e_nn))
    return s, keep


def _opts(alpha, tol, max_iter, fixed_iters, dtype, conv, symmetrize, refine_tol, guess=None, guess_scale=1.0,
          tune=False, graphs=True, progress=False, stop="delta", guard=False):
    return OptsT(float(alpha), float(tol), int(max_iter), int(fixed_iters), _DT[dtype], int(conv),
                 int(symmetrize), float(refine_tol), 0.0, 0, _dev_ptr(guess), float(guess_scale), int(tune),
                 0 if graphs else 1, int(progress), _STOP[stop], int(bool(guard)))


def _records(logs, base, count):
    return [dict(iter=logs[base + k].iter, dtype=logs[base + k].dtype, E=logs[base + k].E, dE=logs[base + k].dE,
                 N=logs[base + k].N, ms=logs[base + k].ms) for k in range(count)]


def scf(ctx: Context, sysd, alpha=0.3, tol=1e-8, max_iter=1000, fixed_iters=0, dtype="f64",
        conv=CONV_AUTO, symmetrize=True, refine_tol=0.0, G_guess=None, want_G=True,
        allow_noconv=False, guess=None, guess_scale=1.0, graphs=True, tune=True, progress=False,
        stop="delta", guard=False, stream=None) -> SCFOut:
    """negf_scf for a workloads.System (guess: learned-guess parameters on the device;
    stop: "delta" or "contraction"; guard: the particle-number guard)."""
    out = scf_batched(ctx, [sysd], alpha=alpha, tol=tol, max_iter=max_iter, fixed_iters=fixed_iters, dtype=dtype,
                      conv=conv, symmetrize=symmetrize, refine_tol=refine_tol,
                      G_guess=None if G_guess is None else [G_guess], want_G=want_G, allow_noconv=allow_noconv,
                      guess=guess, guess_scale=guess_scale, graphs=graphs, tune=tune, single=True,
                      progress=progress, stop=stop, guard=guard, stream=stream)
    return out[0]


def scf_batched(ctx: Context, systems, alpha=0.3, tol=1e-8, max_iter=1000, fixed_iters=0, dtype="f64",
                conv=CONV_AUTO, symmetrize=True, refine_tol=0.0, G_guess=None, want_G=True,
                allow_noconv=False, guess=None, guess_scale=1.0, tune=True, graphs=True, single=False,
                progress=False, stop="delta", guard=False, stream=None):
    """negf_scf_batched (single=True: negf_scf) for a list of workloads.System; returns a list of SCFOut."""
    torch = _torch()
    B = len(systems)
    keep, structs = [], (SystemT * B)()
    for b, sd in enumerate(systems):
        st_, k = system_struct(sd)
        structs[b] = st_
        keep.append(k)
    o = _opts(alpha, tol, max_iter, fixed_iters, dtype, conv, symmetrize, refine_tol, guess, guess_scale, tune,
              graphs, progress, stop, guard)
    Gs = [torch.empty((sd.n_tau, sd.n_b, sd.n_b), dtype=torch.float64, device="cuda") if want_G else None
          for sd in systems]
    Gp = (C.c_void_p * B)(*[_dev_ptr(g) for g in Gs])
    guess_p = None
    if G_guess is not None:
        guess_p = (C.c_void_p * B)(*[_dev_ptr(g) for g in G_guess])
    E, N, hE, hmu = np.zeros(B), np.zeros(B), np.zeros(B), np.zeros(B)
    it, ln = np.zeros(B, dtype=np.int32), np.zeros(B, dtype=np.int32)
    stat = np.zeros(B, dtype=np.int32)
    cap = ((fixed_iters if fixed_iters else max_iter) + max_iter + 4) * (4 if guard else 1)
    logs = (IterLogT * (B * cap))()
    if single:
        rc = lib().negf_scf(ctx.handle, C.byref(structs[0]), C.byref(o), guess_p[0] if guess_p else None,
                            Gp[0], _dptr(E), _dptr(N), it.ctypes.data_as(_IP), logs, cap, _dptr(hE), _dptr(hmu),
                            _stream(stream))
        ln[0] = sum(1 for k in range(cap) if logs[k].ms > 0)
    else:
        rc = lib().negf_scf_batched(ctx.handle, B, structs, C.byref(o), guess_p, Gp, _dptr(E), _dptr(N),
                                    it.ctypes.data_as(_IP), stat.ctypes.data_as(_IP), logs, cap,
                                    ln.ctypes.data_as(_IP), _dptr(hE), _dptr(hmu), _stream(stream))
    if single:
        stat[0] = rc
    if rc != OK and not (allow_noconv and rc in (ENOCONV, ENAN)):
        _check(rc)
    return [SCFOut(Gs[b], float(E[b]), float(N[b]), int(it[b]), float(hE[b]), float(hmu[b]),
                   _records(logs, b * cap, int(ln[b])), int(stat[b])) for b in range(B)]


def matrix_rate(ctx: Context, dtype="f64", stream=None):
    """Measured sustained rate (TFLOP/s) of the matrix-core operation the
    Sigma-2B kernels use for ``dtype``, and the shader clock (GHz) it ran at."""
    tf = C.c_double(0.0)
    ghz = C.c_double(0.0)
    _check(lib().negf_matrix_rate(ctx.handle, _DT[dtype], C.byref(tf), C.byref(ghz), _stream(stream)))
    return tf.value, ghz.value


def f64_issue_probe(ctx: Context, n_mfma, n_fma, stream=None):
    """negf_f64_issue_probe: (ms, MFMA TFLOP/s, vector-FMA TFLOP/s) of a register-only
    loop with n_mfma float64 MFMA chains and n_fma float64 FMA chains per wave."""
    ms, tm, tv = C.c_double(0.0), C.c_double(0.0), C.c_double(0.0)
    _check(lib().negf_f64_issue_probe(ctx.handle, int(n_mfma), int(n_fma), C.byref(ms), C.byref(tm), C.byref(tv),
                                      _stream(stream)))
    return ms.value, tm.value, tv.value


def sigma2b_batched(ctx: Context, Vs, Gs, sigma, dtype="f64", outs=None, stream=None):
    """negf_sigma2b_batched over lists of device tensors V[b] (n_b x n_b), G[b] (n_tau x n_b x n_b)."""
    torch = _torch()
    B = len(Gs)
    if outs is None:
        outs = [torch.empty_like(g) for g in Gs]
    n = np.array([g.shape[1] for g in Gs], dtype=np.int32)
    sg = np.array([sigma] * B if np.isscalar(sigma) else sigma, dtype=np.int32)
    Vp = (C.c_void_p * B)(*[_dev_ptr(v) for v in Vs])
    Gp = (C.c_void_p * B)(*[_dev_ptr(g) for g in Gs])
    Sp = (C.c_void_p * B)(*[_dev_ptr(o) for o in outs])
    _check(lib().negf_sigma2b_batched(ctx.handle, B, n.ctypes.data_as(_IP), int(Gs[0].shape[0]),
                                      sg.ctypes.data_as(_IP), Vp, Gp, Sp, _DT[dtype], _stream(stream)))
    return outs


def sigma2b_batched_set_config(ctx: Context, sizes, dtype, cfg):
    n = np.array(sizes, dtype=np.int32)
    _check(lib().negf_sigma2b_batched_set_config(ctx.handle, len(n), n.ctypes.data_as(_IP), _DT[dtype], int(cfg)))


def sigma2b_batched_tune(ctx: Context, Vs, Gs, sigma, dtype="f64", outs=None, pair_lim=16, stream=None):
    """negf_sigma2b_batched_tune: returns (best config, per-config ms)."""
    torch = _torch()
    B = len(Gs)
    if outs is None:
        outs = [torch.empty_like(g) for g in Gs]
    n = np.array([g.shape[1] for g in Gs], dtype=np.int32)
    sg = np.array([sigma] * B if np.isscalar(sigma) else sigma, dtype=np.int32)
    Vp = (C.c_void_p * B)(*[_dev_ptr(v) for v in Vs])
    Gp = (C.c_void_p * B)(*[_dev_ptr(g) for g in Gs])
    Sp = (C.c_void_p * B)(*[_dev_ptr(o) for o in outs])
    best = C.c_int()
    ms = np.zeros(N_CFG)
    _check(lib().negf_sigma2b_batched_tune(ctx.handle, B, n.ctypes.data_as(_IP), int(Gs[0].shape[0]),
                                           sg.ctypes.data_as(_IP), Vp, Gp, Sp, _DT[dtype], int(pair_lim),
                                           C.byref(best), _dptr(ms), _stream(stream)))
    return best.value, list(ms)


# ------------------------------------------------------------------ learned initial guess
def mlp_param_count() -> int:
    c = C.c_int()
    _check(lib().negf_mlp_param_count(C.byref(c)))
    return c.value


def _nuclei(sysd):
    X = np.ascontiguousarray(sysd.centres, dtype=np.float64).reshape(-1)
    Z = np.ascontiguousarray(sysd.charges, dtype=np.float64).reshape(-1)
    return len(X), X, Z


def mlp_features(ctx: Context, sysd, x_d, v_d, tau_d, ii, jj, qq, stream=None):
    """Feature rows for explicit samples; x_d, v_d, tau_d, ii, jj, qq are device tensors."""
    torch = _torch()
    n_c, X, Z = _nuclei(sysd)
    S = ii.shape[0]
    F = torch.empty((S, 26), dtype=torch.float32, device=x_d.device)
    _check(lib().negf_mlp_features(ctx.handle, sysd.n_b, _dev_ptr(x_d), _dev_ptr(v_d), n_c, _dptr(X), _dptr(Z),
                                   tau_d.shape[0], _dev_ptr(tau_d), float(sysd.beta), S, _dev_ptr(ii),
                                   _dev_ptr(jj), _dev_ptr(qq), _dev_ptr(F), _stream(stream)))
    return F


def mlp_targets(ctx: Context, sysd, x_d, tau_d, G, G0, out_scale, ii, jj, qq, stream=None):
    """Enveloped training targets (G - G0) / (out_scale e) at the samples."""
    torch = _torch()
    n_c, X, Z = _nuclei(sysd)
    S = ii.shape[0]
    t = torch.empty(S, dtype=torch.float32, device=G.device)
    _check(lib().negf_mlp_targets(ctx.handle, G.shape[1], _dev_ptr(G), _dev_ptr(G0), float(out_scale),
                                  _dev_ptr(x_d), n_c, _dptr(X), tau_d.shape[0], _dev_ptr(tau_d), float(sysd.beta), S,
                                  _dev_ptr(ii), _dev_ptr(jj), _dev_ptr(qq), _dev_ptr(t), _stream(stream)))
    return t


def mlp_envelope(ctx: Context, sysd, x_d, tau_d, ii, jj, qq, stream=None):
    torch = _torch()
    n_c, X, Z = _nuclei(sysd)
    S = ii.shape[0]
    e = torch.empty(S, dtype=torch.float32, device=x_d.device)
    _check(lib().negf_mlp_envelope(ctx.handle, _dev_ptr(x_d), n_c, _dptr(X), _dev_ptr(tau_d), float(sysd.beta), S,
                                   _dev_ptr(ii), _dev_ptr(jj), _dev_ptr(qq), _dev_ptr(e), _stream(stream)))
    return e


def mlp_forward(ctx: Context, params, F, stream=None):
    torch = _torch()
    y = torch.empty(F.shape[0], dtype=torch.float32, device=F.device)
    _check(lib().negf_mlp_forward(ctx.handle, _dev_ptr(params), F.shape[0], _dev_ptr(F), _dev_ptr(y),
                                  _stream(stream)))
    return y


def mlp_train_step(ctx: Context, params, m, v, step, lr, F, target, grad_out=None, want_loss=True, stream=None):
    loss = C.c_double()
    _check(lib().negf_mlp_train_step(ctx.handle, _dev_ptr(params), _dev_ptr(m), _dev_ptr(v), int(step), float(lr),
                                     F.shape[0], _dev_ptr(F), _dev_ptr(target), _dev_ptr(grad_out),
                                     C.byref(loss) if want_loss else None, _stream(stream)))
    return loss.value if want_loss else None


def mlp_guess(ctx: Context, params, out_scale, sysd, x_d, v_d, tau_d, G0, G_out=None, dtype="f32", stream=None):
    torch = _torch()
    n_c, X, Z = _nuclei(sysd)
    if G_out is None:
        G_out = torch.empty_like(G0)
    _check(lib().negf_mlp_guess(ctx.handle, _dev_ptr(params), float(out_scale), sysd.n_b, _dev_ptr(x_d),
                                _dev_ptr(v_d), n_c, _dptr(X), _dptr(Z), tau_d.shape[0], _dev_ptr(tau_d),
                                float(sysd.beta), _dev_ptr(G0), _dev_ptr(G_out), _DT[dtype], _stream(stream)))
    return G_out
