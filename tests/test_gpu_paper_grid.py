"""GPU parity on the paper's own case-II grids (Sec. 3.1: 1D He, 29 elements with
n_g = 7, n_b = 202, 200 a.u. box, beta = 100; Sec. 3.2: linear H3+, 13 elements
with n_g = 11, n_b = 142, 50 a.u. box) on short power meshes, so that the
oracle can follow two full second-Born iterations: HF energy, G and the
Galitskii-Migdal energy after two Dyson steps, in float64, to 1e-10."""
import numpy as np
import pytest

import paper_0911_4348_amd as negf
import workloads as W
from oracle import scf as SC

pytestmark = pytest.mark.gpu
TOL64 = 1e-10

CASES = [
    ("he_case2_nb202", W.he_1d(bounds=W.graded_bounds(100.0, 29), n_g=7, beta=100.0).with_(tau_kind="power", u=4, p=3)),
    ("h3p_case2_nb142", W.h3p_1d(R=2.2, bounds=W.graded_bounds(25.0, 13), n_g=11, beta=100.0, tau_kind="power",
                                 u=4, p=3)),
]


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = negf.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("label,s", CASES, ids=[c[0] for c in CASES])
def test_two_iterations_on_the_paper_grid(ctx, label, s):
    print(f"{label}: n_b = {s.n_b}, {s.n_tau} tau points", flush=True)
    ref = SC.scf(s, fixed_iters=2)
    out = negf.scf(ctx, s, fixed_iters=2)
    G = out.G.cpu().numpy()
    err = float(np.max(np.abs(G - ref.G)) / np.max(np.abs(ref.G)))
    print(f"  E_HF {out.hf_E:.10f} (oracle {ref.hf.E + s.e_nn:.10f}), E {out.E:.10f} (oracle {ref.E:.10f}), "
          f"G normwise {err:.1e}", flush=True)
    assert abs(out.hf_E - (ref.hf.E + s.e_nn)) < TOL64 * abs(ref.hf.E)
    assert abs(out.E - ref.E) < TOL64 * abs(ref.E)
    assert err < TOL64
