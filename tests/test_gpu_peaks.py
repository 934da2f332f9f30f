"""Measured-peak helpers of the benchmark (streaming copy and FMA loop)
return plausible figures: below the published MI355X peaks and well above
what a broken launch would give."""
import pytest

pytestmark = pytest.mark.gpu


def test_measured_peaks():
    from paper_1810_07026_amd import airebo
    p = airebo.measured_peaks(copy_mib=256, fma_iters=2048)
    assert 500.0 < p["copy_GBps"] < 8000.0 * 1.05, p          # HBM3E 8 TB/s
    assert 5.0 < p["fp64_fma_TFLOPs"] < 78.6 * 1.05, p         # vector FP64 78.6 TFLOP/s
    assert 5.0 < p["fp32_fma_TFLOPs"] < 157.3 * 1.05, p        # vector FP32 157.3 TFLOP/s (packed)
