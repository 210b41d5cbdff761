"""The SCF's failure paths through the C-ABI (paper Sec. 3.1: the particle
number must stay right during the Dyson iteration; the status codes are the
library's): an iteration cap that is hit, a non-finite start that stops only
its own system, and a learned start with the wrong electron count that is
replaced by the HF start."""
import numpy as np
import pytest

import paper_0911_4348_amd as negf
import workloads as W
from oracle import scf as SC
from paper_0911_4348_amd import learned_guess as LG

pytestmark = pytest.mark.gpu


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


def test_iteration_cap_gives_enoconv_with_valid_outputs(ctx):
    """max_iter = 1: one Dyson step, then NEGF_ENOCONV; G and E are those of the
    first iterate (oracle: exactly one step from G0)."""
    s = W.config_he()
    out = negf.scf(ctx, s, max_iter=1, tol=1e-8, allow_noconv=True)
    assert out.status == negf.ENOCONV
    assert out.iters == 1
    ref = SC.scf(s, fixed_iters=1)
    G = out.G.cpu().numpy()
    assert np.all(np.isfinite(G)) and np.isfinite(out.E) and np.isfinite(out.N)
    assert abs(out.E - ref.E) < 1e-10 * abs(ref.E)
    assert np.max(np.abs(G - ref.G)) < 1e-10 * np.max(np.abs(ref.G))
    with pytest.raises(negf.NegfError) as e:
        negf.scf(ctx, s, max_iter=1, tol=1e-8)
    assert e.value.code == negf.ENOCONV


def test_nan_start_stops_only_its_system(ctx, torch_mod):
    """A batch of two systems; the second starts from a G with one NaN. It ends
    with NEGF_ENAN at its first energy, the first converges as it does alone."""
    torch = torch_mod
    a = W.config_he()
    b = W.random_potential_system(7, W.config_he())
    ga = torch.from_numpy(np.ascontiguousarray(SC.hf_start(a)[2])).cuda()
    gb = torch.from_numpy(np.ascontiguousarray(SC.hf_start(b)[2])).cuda()
    gb[3, 2, 5] = float("nan")
    outs = negf.scf_batched(ctx, [a, b], tol=1e-8, G_guess=[ga, gb], allow_noconv=True)
    assert outs[1].status == negf.ENAN
    assert outs[1].iters == 0
    assert outs[0].status == negf.OK
    alone = negf.scf(ctx, a, tol=1e-8)
    assert outs[0].iters == alone.iters
    assert abs(outs[0].E - alone.E) < 1e-12 * abs(alone.E)
    with pytest.raises(negf.NegfError) as e:
        negf.scf(ctx, b, tol=1e-8, G_guess=gb)
    assert e.value.code == negf.ENAN


def test_learned_start_with_wrong_electron_count_falls_back_to_hf_start(ctx, torch_mod):
    """The shipped network with its output scaled up 1e4-fold gives a start whose
    electron count -sigma Tr G(beta^-) is far from 2; the library must replace it
    by G0, so the run is the HF-started one: same steps, same energy."""
    torch = torch_mod
    p, scale, _ = LG.load()
    P = torch.from_numpy(p).cuda()
    s = W.random_potential_system(100003)
    x, Wt, T, v, V = negf.fedvr_build_system(s)
    tau = negf.tau_grid_system(s)
    hfs = negf.hf(ctx, torch.from_numpy(T).cuda(), torch.from_numpy(v).cuda(), torch.from_numpy(V).cuda(),
                  s.n_elec, s.sigma, s.beta)
    G0 = negf.g0_build(ctx, hfs, tau, s.beta)
    bad = negf.mlp_guess(ctx, P, 1e4 * scale, s, torch.from_numpy(x).cuda(), torch.from_numpy(v).cuda(),
                         torch.from_numpy(tau).cuda(), G0, dtype="bf16")
    N_bad = -s.sigma * float(torch.trace(bad[-1]))
    print(f"electron count of the inflated learned start: {N_bad:.4f}")
    assert not abs(N_bad - s.n_elec) <= 0.02 * s.n_elec
    hf_run = negf.scf(ctx, s, tol=1e-6, conv=negf.CONV_FFT, want_G=False)
    lg_run = negf.scf(ctx, s, tol=1e-6, conv=negf.CONV_FFT, want_G=False, guess=P, guess_scale=1e4 * scale)
    assert lg_run.status == negf.OK
    assert lg_run.iters == hf_run.iters
    assert lg_run.E == hf_run.E


def test_contraction_stop_matches_oracle(ctx):
    """The contraction-aware stopping rule stops at the same step as the oracle's."""
    s = W.config_he()
    ref = SC.scf(s, tol=1e-7, stop="contraction")
    out = negf.scf(ctx, s, tol=1e-7, stop="contraction")
    print(f"contraction rule: {out.iters} steps (oracle {ref.iters}), E = {out.E:.12f}")
    assert out.status == negf.OK and out.iters == ref.iters
    assert abs(out.E - ref.E) < 1e-10 * abs(ref.E)


def test_guard_restart_matches_oracle(ctx, torch_mod):
    """Runaway guard: a start with a quarter of the electrons is replaced by G0 with
    alpha halved, in the library as in the oracle (same steps, same result)."""
    s = W.config_he()
    setup, hf, G0 = SC.hf_start(s)
    ref = SC.scf(s, alpha=0.3, tol=1e-8, G_init=0.25 * G0, guard=True, setup=setup, hf=hf)
    g = torch_mod.from_numpy(np.ascontiguousarray(0.25 * G0)).cuda()
    out = negf.scf(ctx, s, alpha=0.3, tol=1e-8, G_guess=g, guard=True)
    print(f"guard: {out.iters} steps (oracle {ref.iters}, {ref.backoffs} restart)")
    assert ref.backoffs == 1 and out.status == negf.OK and out.iters == ref.iters
    assert abs(out.E - ref.E) < 1e-10 * abs(ref.E)
    assert np.max(np.abs(out.G.cpu().numpy() - ref.G)) < 1e-9 * np.max(np.abs(ref.G))


def test_density_at_nodes_matches_oracle(ctx, torch_mod):
    """negf_density on an SCF iterate: n(x_a) = -sigma G_aa(beta^-) / W_a."""
    from oracle import observables as O
    s = W.config_he()
    ref = SC.scf(s, fixed_iters=3)
    out = negf.scf(ctx, s, fixed_iters=3)
    x, Wt, T, v, V = negf.fedvr_build_system(s)
    n = negf.density(ctx, torch_mod.from_numpy(Wt).cuda(), out.G, 2).cpu().numpy()
    nref = O.density_nodes(ref.G, ref.setup.W, 2)
    assert np.max(np.abs(n - nref)) < 1e-10 * np.max(nref)
    n32 = negf.density(ctx, torch_mod.from_numpy(Wt).cuda(), out.G.float(), 2, dtype="f32").cpu().numpy()
    assert np.max(np.abs(n32 - nref)) < 1e-6 * np.max(nref)
