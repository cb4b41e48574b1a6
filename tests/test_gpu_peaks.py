"""Measured device peaks (the roofline denominators the bench reports beside
the vendor figures): each microbenchmark returns a rate between a tenth of
and the vendor peak of the part (FP64 vector and MFMA 78.6 TFLOP/s, HBM
8 TB/s), through the C ABI."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_05087_amd as F  # noqa: E402


def test_measured_peaks_are_plausible():
    p = F.fmddm_measure_peaks()
    print(p)
    assert 7.86 <= p["fp64_vector_tflops"] <= 78.6 * 1.02
    assert 7.86 <= p["fp64_mfma_tflops"] <= 78.6 * 1.02
    assert 800.0 <= p["copy_gbps"] <= 8000.0 * 1.02
