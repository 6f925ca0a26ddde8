"""Measured ceilings of the GPU the stem kernels run on (C-ABI stem_mb_*):
streaming copy bandwidth from HBM and from the 256 MiB last-level cache,
and the dense MFMA rates of the product kernels' instruction shapes."""

from __future__ import annotations

import ctypes

from . import _capi as C
from .stem import _stream_handle


def _time(fn, reps: int) -> float:
    import torch

    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def copy_gbs(nbytes: int, vec_bytes: int = 16, blocks: int = 8192, reps: int = 10) -> float:
    """Read + write bytes per second of a device copy of nbytes."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    st = _stream_handle(None)

    def run():
        C.check(C.lib().stem_mb_copy(ctypes.c_void_p(src.data_ptr()),
                                     ctypes.c_void_p(dst.data_ptr()), nbytes, vec_bytes, blocks,
                                     st))

    t = _time(run, reps)
    return 2 * nbytes / t / 1e9


def mfma_tflops(kind: int, iters: int = 4096, blocks: int = 4096) -> float:
    """Dense rate of one MFMA kind (0 f32 16x16x4, 1 f16 16x16x32, 2 bf16 16x16x32)."""
    import torch

    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    st = _stream_handle(None)

    def run():
        C.check(C.lib().stem_mb_mfma(kind, iters, blocks, ctypes.c_void_p(out.data_ptr()), st))

    t = _time(run, 3)
    per = 2048.0 if kind == 0 else 16384.0
    waves = blocks * 4
    return waves * 8 * iters * per / t / 1e12


def measure() -> dict:
    return {
        "hbm_copy_gbs_16B": round(copy_gbs(4 << 30, 16), 1),
        "hbm_copy_gbs_8B": round(copy_gbs(4 << 30, 8), 1),
        "llc_copy_gbs_16B": round(copy_gbs(64 << 20, 16, reps=50), 1),
        "mfma_f32_tflops": round(mfma_tflops(0), 1),
        "mfma_f16_tflops": round(mfma_tflops(1), 1),
        "mfma_bf16_tflops": round(mfma_tflops(2), 1),
    }
