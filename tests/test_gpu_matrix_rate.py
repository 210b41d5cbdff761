"""Measured matrix-core ceiling (negf_matrix_rate): the rate of the MFMA shape
the Sigma-2B kernels issue, reported beside the datasheet peak in the bench
line. Checks that it runs, that the clock it reports is a plausible shader
clock, and that no rate exceeds what that clock allows for the datasheet's
per-cycle throughput (MI355X: 256 CUs, 78.6 / 157.3 / 2500 TFLOP/s dense at
2.4 GHz for float64 / float32 / bf16)."""
import pytest

import paper_0911_4348_amd as negf

pytestmark = pytest.mark.gpu

PEAK_AT_2400MHZ = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = negf.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_matrix_rate_bounded_by_clock(ctx, dtype):
    tf, ghz = negf.matrix_rate(ctx, dtype)
    print(f"{dtype}: {tf:.1f} TFLOP/s at {ghz:.3f} GHz")
    assert 0.5 < ghz < 3.0
    assert tf > 0.0
    assert tf <= PEAK_AT_2400MHZ[dtype] * ghz / 2.4 * 1.05


def test_matrix_rate_rejects_bad_dtype(ctx):
    with pytest.raises(KeyError):
        negf.matrix_rate(ctx, "f16")


def test_issue_probe_runs_and_stays_below_peak(ctx):
    """negf_f64_issue_probe: every built combination runs and reports rates that the
    float64 datasheet peak bounds; an unbuilt combination is refused."""
    for nm, nv in ((8, 0), (0, 8), (8, 8)):
        ms, tm, tv = negf.f64_issue_probe(ctx, nm, nv)
        print(f"{nm} MFMA, {nv} FMA chains: {ms:.3f} ms, {tm:.1f} + {tv:.1f} TFLOP/s")
        assert ms > 0.0
        assert (tm > 0.0) == (nm > 0) and (tv > 0.0) == (nv > 0)
        assert tm + tv <= PEAK_AT_2400MHZ["f64"] * 1.05
    with pytest.raises(negf.NegfError):
        negf.f64_issue_probe(ctx, 4, 4)
