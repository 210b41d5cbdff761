"""The bond-length scan of linear H3+ at its full sizes (R = 1..3, n_b = 149..399,
1025 tau points, beta = 100): the HF energy curve against the oracle instance by
instance, and the persistent Sigma-2B launch over uneven instances on sampled
slices against the oracle."""
import numpy as np
import pytest

import paper_0911_4348_amd as negf
import workloads as W
from oracle import fedvr, hf as H, sigma as S

pytestmark = pytest.mark.gpu
TOL64 = 1e-10


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


def test_scan_hf_curve_matches_oracle(ctx, torch_mod):
    systems = W.config_scan()[::8]
    d = lambda a: torch_mod.from_numpy(np.ascontiguousarray(a)).cuda()
    for s in systems:
        print(f"scan HF R={s.centres[2]:.3f} n_b={s.n_b}", flush=True)
        x, Wt, T, v, V = negf.fedvr_build_system(s)
        hfs = negf.hf(ctx, d(T), d(v), d(V), 2.0, 2, s.beta)
        st = fedvr.Setup(s)
        o = H.hartree_fock(st.h, st.V, 2.0, 2, s.beta)
        assert abs(hfs.E - o.E) < TOL64 * abs(o.E), s.centres[2]


def test_scan_sigma2b_batched_full_size_sampled(ctx, torch_mod):
    """Four scan instances (smallest, two middle, largest) in one persistent launch;
    G_q = A e^(-tau_q/4) + B e^(-(beta - tau_q)/4) with seeded symmetric A, B per instance."""
    torch = torch_mod
    scan = W.config_scan()
    picks = [scan[0], scan[21], scan[42], scan[63]]
    Vs, Gs, AB = [], [], []
    for k, s in enumerate(picks):
        x, Wt, T, v, V = negf.fedvr_build_system(s)
        tau = negf.tau_grid_system(s)
        A = W.random_symmetric(s.n_b, 40 + k, 0.1)
        B = W.random_symmetric(s.n_b, 50 + k, 0.1)
        a = torch.from_numpy(np.exp(-tau / 4.0)).cuda()[:, None, None]
        b = torch.from_numpy(np.exp(-(s.beta - tau) / 4.0)).cuda()[:, None, None]
        Gs.append((torch.from_numpy(A).cuda()[None] * a + torch.from_numpy(B).cuda()[None] * b).contiguous())
        Vs.append(torch.from_numpy(V).cuda())
        AB.append((V, A, B, np.exp(-tau / 4.0), np.exp(-(s.beta - tau) / 4.0)))
    print("scan sigma2b batched sizes", [s.n_b for s in picks], flush=True)
    outs = negf.sigma2b_batched(ctx, Vs, Gs, 2)
    torch.cuda.synchronize()
    n_tau = picks[0].n_tau
    for (V, A, B, a, b), o in zip(AB, outs):
        for q in (3, 700):
            Gq = A * a[q] + B * b[q]
            Gb = A * a[n_tau - 1 - q] + B * b[n_tau - 1 - q]
            ref = S.sigma2b_slice(V, Gq, Gb, 2)
            got = o[q].cpu().numpy()
            assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < TOL64, (V.shape, q)
