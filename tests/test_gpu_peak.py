"""The FP64 FMA throughput measurement (amiMeasureFp64Peak) on the GPU: a
positive rate no higher than the device's FP64 vector peak allows, and its
argument checks."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amd = pytest.importorskip("paper_2311_17189_amd")


def test_measured_fp64_peak():
    tf = amd.measure_fp64_peak(1 << 12)
    # 256 CUs x 128 FP64 FLOP per clock at most 2.4 GHz: 78.6 TFLOP/s
    assert 1.0 < tf <= 78.6 * 1.05, tf
    for bad in (0, (1 << 24) + 1):
        with pytest.raises(amd.AmiError) as e:
            amd.measure_fp64_peak(bad)
        assert e.value.code == -1
