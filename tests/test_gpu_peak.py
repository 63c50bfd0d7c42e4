"""The attainable-MFMA-rate diagnostic (afqmc_mfma_peak): a positive rate no higher than the
datasheet peak of the instruction family, and about the same on a repeat."""

import pytest

pytestmark = pytest.mark.gpu

DATASHEET = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0}   # TFLOP/s, dense


@pytest.mark.parametrize("precision", list(DATASHEET))
def test_mfma_peak_is_below_the_datasheet(precision):
    import paper_1711_02242_amd as afq
    from tests.parity_helpers import log
    a = afq.mfma_peak(precision)
    b = afq.mfma_peak(precision)
    log(f"mfma peak {precision}: {a:.1f}, {b:.1f} TFLOP/s (datasheet {DATASHEET[precision]})")
    assert 0.3 * DATASHEET[precision] < a <= 1.02 * DATASHEET[precision]
    assert abs(a - b) < 0.15 * a
