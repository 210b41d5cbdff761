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
