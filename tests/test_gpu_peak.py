"""The FP32 FMA-rate measurement aid runs and gives a plausible figure: below
the published packed peak (157.3 TFLOP/s) and above a tenth of the unpacked
one (78.6 TFLOP/s)."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_valu_fma_rate_is_plausible():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2512_11571_amd import binding
    r = binding.valu_fma_rate() / 1e12
    assert 7.86 < r < 157.3, r
