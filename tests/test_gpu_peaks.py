"""The measured ceilings (include/bsm_peaks.h) on the GPU: each probe's
rate must lie between 30 % and 105 % of the published MI355X figure of its
unit.  Above it, the probe's operation or byte count would be wrong; far
below it, the probe would not be exercising the unit it names."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch

PUBLISHED = {
    # 256 CUs x 2.4 GHz x 64 lanes: one unpacked lane operation per lane
    # and clock (the rate behind the 78.6 TFLOP/s fp64 vector figure)
    "valu_int32_ops": 256 * 64 * 2.4e9,
    # adds and xors issue faster, at most at the packed rate behind the
    # 157.3 TFLOP/s fp32 vector figure (128 per CU and clock)
    "valu_addxor_ops": 256 * 128 * 2.4e9,
    # dense int8 matrix operations per second
    "mfma_i8_ops": 5.0e15,
    # dense fp4 (e2m1) matrix operations per second
    "mfma_fp4_ops": 10.1e15,
    # HBM3E
    "hbm_read_bps": 8.0e12,
    "hbm_copy_bps": 8.0e12,
}


def test_measured_peaks_are_plausible(torch_cuda):
    from paper_1402_2020_amd import _bsm
    p = _bsm.bsm_measure_peaks(0, 1 << 30, 2)
    print({k: (f"{v:.4g}" if isinstance(v, float) else v) for k, v in p.items()})
    assert p["compute_units"] >= 1
    for key, ref in PUBLISHED.items():
        assert 0.3 * ref <= p[key] <= 1.05 * ref, (key, p[key], ref)


def test_measure_peaks_rejects_an_unknown_device(torch_cuda):
    from paper_1402_2020_amd import _bsm
    with pytest.raises(_bsm.BsmError):
        _bsm.bsm_measure_peaks(1 << 20, 1 << 30, 1)
