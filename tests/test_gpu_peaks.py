"""Measured device peaks (``include/adg_peaks.h``): the rates are positive and
within physical bounds of the published figures (FP64 vector and matrix
78.6 TFLOP/s, HBM 8 TB/s), and the copy moved the data."""
import pytest

torch = pytest.importorskip("torch")

from paper_1905_05524_amd import adg

pytestmark = pytest.mark.gpu


def test_measured_peaks_are_plausible():
    p = adg.measure_peaks(copy_mib=256)
    assert 5.0 < p["fp64_vector_tflops"] < 1.2 * p["fp64_vector_tflops_spec"], p
    assert 5.0 < p["fp64_mfma_tflops"] < 1.2 * p["fp64_mfma_tflops_spec"], p
    # a 256 MiB copy may run partly from the 256 MB last-level cache
    assert 300.0 < p["copy_GBps"] < 3.0 * p["hbm_GBps_spec"], p


def test_peaks_reject_misaligned_copy():
    nb = adg.ctypes.c_size_t()
    adg._check(adg.lib().adg_peaks_sink_bytes(adg.ctypes.byref(nb)))
    sink = torch.empty(nb.value // 8, dtype=torch.float64, device="cuda")
    src = torch.ones(1024, dtype=torch.float64, device="cuda")
    out = (adg.ctypes.c_double * 3)()
    rc = adg.lib().adg_measure_peaks(adg.ctypes.c_void_p(sink.data_ptr()), adg.ctypes.c_void_p(src.data_ptr()),
                                     adg.ctypes.c_void_p(src.data_ptr() + 8), 8000, out, None)
    assert rc == adg.ADG_EINVAL
