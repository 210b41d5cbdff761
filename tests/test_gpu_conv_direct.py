"""GPU parity of the Dyson step on the direct-quadrature route (negf_dyson_step
with CONV_DIRECT) against the float64 oracle, whole tensor, at the sizes that
select every launch shape of the strip kernel: one and several 64-row strips,
every column-tile template, and more than one column launch (paper Sec. 2.3,
Eq. deq; the power mesh of Sec. 3.1).

The step is linear in Sigma_c and accepts any symmetric G, so G = G0 plus a
seeded symmetric perturbation and a seeded symmetric Sigma_c stand in for an
SCF iterate and its second-Born self-energy (an oracle Sigma-2B evaluation at
n_b = 359 would cost minutes of CPU time and test nothing more here).

Bar: float64 normwise relative error <= 1e-10 (max |gpu - oracle| / max
|oracle| over the whole tensor); the float32 step states its error."""
import numpy as np
import pytest

import paper_0911_4348_amd as negf
import workloads as W
from oracle import fedvr, dyson as D, scf as SC

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx(torch_mod):
    c = negf.Context(0)
    yield c
    c.close()


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _case(s, seed):
    """HF of system s (oracle), and seeded symmetric inputs G, Sigma_c of its size."""
    setup, o = SC.run_hf(s)
    kind = "power" if s.tau_kind == "power" else "uniform"
    dctx = D.DysonContext(setup, o, kind, block=s.u if kind == "power" else 0)
    n_t, n = dctx.G0.shape[0], setup.h.shape[0]
    G = dctx.G0 + 0.02 * W.random_symmetric_slices(n, n_t, seed)
    Sc = 0.01 * W.random_symmetric_slices(n, n_t, seed + 1)
    return setup, o, dctx, G, Sc


# (label, system, expected strip-kernel column template, column launches)
CASES = [
    ("h3p_nb359_power_u8p4",
     W.config_h3p().with_(u=8, p=4), 13, 1),
    ("nb429_power_u4p3",
     W.he_1d(half_width=43.0, n_e=86, n_g=5, beta=20.0).with_(tau_kind="power", u=4, p=3), 13, 2),
    ("he_nb199_uniform_M64",
     W.config_sigma_bench().with_(M=64), 7, 1),
    ("he_nb99_uniform_M32",
     W.he_1d(half_width=20.0, n_e=20, n_g=5, beta=20.0, M=32), 4, 1),
]


def _launch_shape(n):
    """Column template and number of column launches the library picks for n
    (the rule of the strip kernel's launcher, restated to label the case)."""
    jtw = ((n + 15) // 16 + 1) // 2
    jt = 2 if jtw <= 2 else 4 if jtw <= 4 else 7 if jtw <= 7 else 13
    return jt, -(-n // (2 * jt * 16))


@pytest.mark.parametrize("label,s,jt,launches", CASES, ids=[c[0] for c in CASES])
def test_dyson_direct_route_whole_tensor(ctx, torch_mod, label, s, jt, launches):
    n = s.n_b
    assert _launch_shape(n) == (jt, launches)
    print(f"dyson CONV_DIRECT {label}: n_b={n}, {s.n_tau} tau points, {(n + 63) // 64} strips, "
          f"template {jt}, {launches} column launch(es)", flush=True)
    setup, o, dctx, G, Sc = _case(s, 500 + n)
    x, Wt, T, v, V = negf.fedvr_build_system(s)
    hfs = negf.hf(ctx, dev(torch_mod, T), dev(torch_mod, v), dev(torch_mod, V), s.n_elec, s.sigma, s.beta)
    tg = negf.TauGrid.of_system(s)
    h = T + np.diag(v)
    Gout, E, N = negf.dyson_step(ctx, tg, s.sigma, dev(torch_mod, h), dev(torch_mod, V), hfs, dev(torch_mod, G),
                                 dev(torch_mod, Sc), 0.3, conv=negf.CONV_DIRECT)
    got = Gout.cpu().numpy()
    ref = D.dyson_step(dctx, G, Sc, 0.3, route="direct")
    err = relerr(got, ref)
    Eref = D.gm_energy(setup.h, setup.V, s.sigma, G, Sc, setup.tau)
    print(f"  float64: normwise error {err:.2e}, |E - E_oracle| = {abs(E - Eref):.2e} Ha", flush=True)
    assert err < TOL64
    assert abs(E - Eref) < TOL64 * abs(Eref)
    assert abs(N - D.particle_number(G, s.sigma)) < 1e-11
    f32 = torch_mod.float32
    G32, E32, _ = negf.dyson_step(ctx, tg, s.sigma, dev(torch_mod, h), dev(torch_mod, V), hfs,
                                  dev(torch_mod, G, f32), dev(torch_mod, Sc, f32), 0.3, conv=negf.CONV_DIRECT,
                                  dtype="f32")
    err32 = relerr(G32.double().cpu().numpy(), ref)
    print(f"  float32: normwise error {err32:.2e}, |E - E_oracle| = {abs(E32 - Eref):.2e} Ha", flush=True)
    assert err32 < 1e-5
    assert abs(E32 - Eref) < 1e-5 * abs(Eref)
