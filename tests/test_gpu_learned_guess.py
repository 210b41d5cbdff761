"""What the trained network gains: on held-out random potentials (the learned-
guess workload: n_b = 199, 1025 tau points, beta = 50) the SCF started from
G0 + the network's correction reaches |E - E_ref| < 1e-6 Ha in fewer steps than
the HF start, and both starts converge to the same energy."""
import os

import numpy as np
import pytest

import paper_0911_4348_amd as negf
import workloads as W
from paper_0911_4348_amd import learned_guess as LG

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _steps_to(log, E_ref, tol=1e-6):
    for k, r in enumerate(log):
        if abs(r["E"] - E_ref) < tol:
            return k
    return len(log)


def test_trained_weights_are_shipped():
    assert os.path.exists(LG.WEIGHTS)
    p, scale, info = LG.load()
    assert p.size == negf.mlp_param_count() and np.all(np.isfinite(p)) and scale > 0
    assert info["history"][-1]["val_rel"] < 0.5


def test_learned_start_saves_steps_at_equal_energy(torch_mod):
    torch = torch_mod
    ctx = negf.Context(0)
    p, scale, _ = LG.load()
    P = torch.from_numpy(p).cuda()
    hf_steps, lg_steps = [], []
    for seed in (100000, 100007, 100016):
        print(f"learned guess seed {seed}", flush=True)
        s = W.random_potential_system(seed)
        a = negf.scf(ctx, s, tol=1e-8, conv=negf.CONV_FFT, want_G=False, max_iter=400)
        b = negf.scf(ctx, s, tol=1e-8, conv=negf.CONV_FFT, want_G=False, max_iter=400, guess=P, guess_scale=scale)
        assert abs(a.E - b.E) < 2e-7, (seed, a.E, b.E)      # same fixed point
        hf_steps.append(_steps_to(a.log, a.E))
        lg_steps.append(_steps_to(b.log, a.E))
        print(f"  steps to 1e-6 Ha: HF start {hf_steps[-1]}, learned start {lg_steps[-1]}")
    assert sum(lg_steps) < sum(hf_steps)
    ctx.close()
