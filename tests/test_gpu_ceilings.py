"""Ceiling microbenchmarks run and give physically sensible rates: the copy
moves its bytes correctly and no measured rate exceeds the datasheet peak
(8 TB/s HBM; 157.3 TFLOP/s FP32 and 2.5 PFLOP/s FP16/BF16 dense MFMA)."""
import ctypes

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2005_06787_amd import _capi as C  # noqa: E402
from paper_2005_06787_amd import ceilings  # noqa: E402


@pytest.mark.parametrize("vec", [8, 16])
def test_copy_is_exact(vec):
    n = (1 << 20) + 16
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    C.check(C.lib().stem_mb_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                 4 * n, vec, 64, None))
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_ceilings_within_datasheet():
    c = ceilings.measure()
    print(c)
    assert 1000 < c["hbm_copy_gbs_16B"] <= 8000 * 1.02
    assert 1000 < c["hbm_copy_gbs_8B"] <= 8000 * 1.02
    assert 20 < c["mfma_f32_tflops"] <= 157.3 * 1.02
    assert 200 < c["mfma_f16_tflops"] <= 2500 * 1.02
    assert 200 < c["mfma_bf16_tflops"] <= 2500 * 1.02
