"""negf_sigma2b_noalloc (the allocation-free Sigma-2B entry point) against
negf_sigma2b through the C-ABI: bitwise-equal output (same kernels, same tile
configuration), in float64 and float32, on two calls in a row, the second
smaller; no scratch allocated in the context that makes the calls; host-side
rejection of sizes beyond the fixed array and of bf16."""
import ctypes as C

import numpy as np
import pytest

import paper_0911_4348_amd as negf
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _inputs(torch, n, n_tau, seed, dt):
    V = np.abs(W.random_symmetric(n, seed)) + 0.1
    G = W.random_symmetric_slices(n, n_tau, seed + 1)
    return torch.from_numpy(V).to("cuda", dt), torch.from_numpy(G).to("cuda", dt)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_sigma2b_on_two_calls(torch_mod, dtype):
    torch = torch_mod
    dt = torch.float64 if dtype == "f64" else torch.float32
    ref_ctx = negf.Context(0)
    na_ctx = negf.Context(0)
    try:
        for n, n_tau, seed in ((45, 11, 3), (21, 6, 9)):      # the second call is smaller
            print(f"noalloc {dtype} n_b={n} n_tau={n_tau}", flush=True)
            V, G = _inputs(torch, n, n_tau, seed, dt)
            ref = negf.sigma2b(ref_ctx, V, G, 2, dtype=dtype)
            out = torch.full_like(G, float("nan"))
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            negf.sigma2b_noalloc(na_ctx, V, G, 2, out, dtype=dtype)
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == before
            assert na_ctx.scratch_bytes() == 0
            assert torch.equal(out, ref), float((out - ref).abs().max())
    finally:
        ref_ctx.close()
        na_ctx.close()


def test_noalloc_rejects_what_it_cannot_hold(torch_mod):
    torch = torch_mod
    ctx = negf.Context(0)
    try:
        V, G = _inputs(torch, 8, 3, 1, torch.float32)
        out = torch.empty_like(G)
        with pytest.raises(negf.NegfError) as e:
            negf.sigma2b_noalloc(ctx, V, G, 2, out, dtype="bf16")
        assert e.value.code == negf.EINVAL
        L = negf.lib()
        rc = L.negf_sigma2b_noalloc(ctx.handle, 8, 65537, 2, C.c_void_p(V.data_ptr()), C.c_void_p(G.data_ptr()),
                                    C.c_void_p(out.data_ptr()), negf.F32, None)
        assert rc == negf.EINVAL and b"allocation-free" in L.negf_last_error()
        assert ctx.scratch_bytes() == 0
    finally:
        ctx.close()
