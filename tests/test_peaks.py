"""The peak microbenchmarks behind the roofline denominators run and return
rates of the right magnitude: each within a factor of the chip's published
figure (FP64 vector 78.6 TFLOP/s, dense bf16 2.5 PFLOP/s, HBM 8 TB/s), never
above it by more than timing noise.  Unpacked FP32 FMA (one operation per
instruction) is bounded by the same issue rate as FP64: the published 157.3
TFLOP/s FP32 vector figure needs packed instructions."""

import pytest

pytestmark = pytest.mark.gpu


def test_measured_peaks_are_near_the_published_ones():
    from paper_1501_03450_amd import binding as B
    pk = B.st_measure_peaks(0)
    print(pk)
    assert 0.3 * 78.6 < pk["fp64_fma_tflops"] < 1.05 * 78.6
    assert 0.3 * 78.6 < pk["fp32_fma_tflops"] < 1.05 * 78.6
    assert 0.2 * 2500.0 < pk["bf16_mfma_tflops"] < 1.05 * 2500.0
    assert 0.2 * 8000.0 < pk["copy_gbps"] < 1.05 * 8000.0
