"""The roofline probes (measurement, not part of the method) report rates that the GPU can reach:
positive and within the datasheet's ceilings (HBM 8 TB/s over buffers of 2 GiB, eight times the
memory-side cache; FP64 matrix cores 78.6 TFLOP/s, FP32 157.3), with 5% allowance for clocks."""
import pytest

from gpu_helpers import print_case

pytestmark = pytest.mark.gpu


def test_bandwidth_probes_within_hbm_peak():
    from paper_0901_3512_amd import probe_bandwidth
    for kind in ("copy", "triad", "read"):
        print_case("probe", kind)
        gbs = probe_bandwidth(kind, 1 << 31, 5)
        print(kind, gbs)
        assert 1000.0 < gbs <= 8000.0 * 1.05, (kind, gbs)


def test_mfma_probes_within_matrix_peak():
    from paper_0901_3512_amd import probe_mfma
    for dtype, peak in (("fp64", 78.6), ("fp32", 157.3)):
        print_case("probe mfma", dtype)
        tf = probe_mfma(dtype, 5000)
        print(dtype, tf)
        assert 5.0 < tf <= peak * 1.05, (dtype, tf)


def test_probes_refuse_bad_arguments():
    from paper_0901_3512_amd import SeedCGError, probe_bandwidth, probe_mfma
    with pytest.raises(KeyError):
        probe_bandwidth("scale")
    with pytest.raises(SeedCGError):
        probe_bandwidth("copy", 1024)
    with pytest.raises(SeedCGError):
        probe_mfma("fp64", 0)
