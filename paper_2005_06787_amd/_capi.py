"""ctypes declarations of libstemgpu's C-ABI (include/stemgpu.h).

Argument marshalling only.  The library is loaded from this package's
``_lib/`` folder; if it is not there the import fails with a message that
says how to build it -- there is no other implementation to fall back on.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libstemgpu.so")

STEM_OK = 0
STEM_EINVAL = 1
STEM_ELABEL = 2
STEM_ESHAPE = 3
STEM_EUNSUPPORTED = 4
STEM_ENOMEM = 5
STEM_ERANGE = 6
STEM_EHIP = 7

STEM_FP32 = 0
STEM_SPLIT_FP16 = 1
STEM_SPLIT_BF16 = 2

STEM_ACCUMULATE = 1
STEM_TIME_STEPS = 2

PRECISIONS = {"fp32": STEM_FP32, "split_fp16": STEM_SPLIT_FP16, "split_bf16": STEM_SPLIT_BF16}

_i32p = ctypes.POINTER(ctypes.c_int32)
_f32p = ctypes.POINTER(ctypes.c_float)


class stem_plan_desc(ctypes.Structure):
    _fields_ = [
        ("n_open", ctypes.c_int32), ("open_labels", _i32p),
        ("n_sliced", ctypes.c_int32), ("sliced_labels", _i32p),
        ("n_proj", ctypes.c_int32), ("proj_labels", _i32p),
        ("stem_rank", ctypes.c_int32), ("stem_labels", _i32p),
        ("stem_data", ctypes.c_void_p), ("stem_on_device", ctypes.c_int32),
        ("n_branches", ctypes.c_int32), ("branch_ranks", _i32p),
        ("branch_labels", _i32p), ("branch_data", ctypes.c_void_p),
        ("precision", ctypes.c_int32), ("max_rank", ctypes.c_int32),
    ]


class stem_step_info(ctypes.Structure):
    _fields_ = [
        ("rank_in", ctypes.c_int32), ("rank_out", ctypes.c_int32),
        ("n_shared", ctypes.c_int32), ("n_free", ctypes.c_int32),
        ("permuted", ctypes.c_int32), ("last_slices", ctypes.c_int32),
        ("M", ctypes.c_int64), ("K", ctypes.c_int64), ("N", ctypes.c_int64),
        ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
        ("perm_bytes", ctypes.c_double),
        ("last_gemm_us", ctypes.c_float), ("last_perm_us", ctypes.c_float),
        ("amode", ctypes.c_int32), ("cmode", ctypes.c_int32),
        ("sched_tm", ctypes.c_int32), ("sched_ntw", ctypes.c_int32),
        ("sched_blocks", ctypes.c_int32), ("sched_lds", ctypes.c_int32),
        ("tuned_us", ctypes.c_float), ("tuned_slices", ctypes.c_int32),
        ("n_batch", ctypes.c_int32), ("sched_algo", ctypes.c_int32),
    ]


class stem_plan_summary(ctypes.Structure):
    _fields_ = [
        ("n_steps", ctypes.c_int32), ("peak_rank", ctypes.c_int32),
        ("n_permutes", ctypes.c_int32), ("n_open", ctypes.c_int32),
        ("flops_per_slice", ctypes.c_double), ("bytes_per_slice", ctypes.c_double),
        ("perm_bytes_per_slice", ctypes.c_double), ("n_slices", ctypes.c_uint64),
    ]


class stem_hw(ctypes.Structure):
    _fields_ = [
        ("hbm_bytes_per_s", ctypes.c_double), ("fp32_flops_per_s", ctypes.c_double),
        ("fp16_flops_per_s", ctypes.c_double), ("launch_s", ctypes.c_double),
    ]


STEM_N_FEATURES = 12
_f32p_ = ctypes.POINTER(ctypes.c_float)

# name -> (restype, argtypes); every function declared in include/stemgpu.h
SIGNATURES = {
    "stem_plan_steps": (ctypes.c_int32, [ctypes.POINTER(stem_plan_desc),
                                         ctypes.POINTER(stem_step_info), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "stem_cost_analytic": (ctypes.c_int32, [ctypes.POINTER(stem_step_info), ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                                            ctypes.POINTER(stem_hw),
                                            ctypes.POINTER(ctypes.c_double)]),
    "stem_step_features": (ctypes.c_int32, [ctypes.POINTER(stem_step_info), ctypes.c_int32,
                                            ctypes.c_uint32, _f32p_]),
    "stem_mlp_n_params": (ctypes.c_int64, [ctypes.c_int32, ctypes.c_int32]),
    "stem_mlp_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, _f32p_,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "stem_mlp_set_scaling": (ctypes.c_int32, [ctypes.c_void_p, _f32p_, _f32p_, ctypes.c_float,
                                              ctypes.c_float]),
    "stem_mlp_get_params": (ctypes.c_int32, [ctypes.c_void_p, _f32p_]),
    "stem_mlp_loss_grad": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "stem_mlp_train": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "stem_mlp_predict": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "stem_mlp_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "stem_mb_copy": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "stem_mb_mfma": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "stem_plan_validate": (ctypes.c_int32, [ctypes.POINTER(stem_plan_desc),
                                            ctypes.POINTER(stem_plan_summary)]),
    "stem_plan_create": (ctypes.c_int32, [ctypes.POINTER(stem_plan_desc), ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "stem_plan_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "stem_plan_summary_get": (ctypes.c_int32, [ctypes.c_void_p,
                                               ctypes.POINTER(stem_plan_summary)]),
    "stem_plan_workspace_bytes": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32,
                                                   ctypes.POINTER(ctypes.c_uint64)]),
    "stem_step_info_get": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.POINTER(stem_step_info)]),
    "stem_contract": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint32,
                                       ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                       ctypes.c_uint32, ctypes.c_void_p]),
    "stem_tune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.c_uint64, ctypes.c_int32, ctypes.c_char_p,
                                   ctypes.c_void_p]),
    "stem_batch_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                                           ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "stem_batch_launch": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "stem_batch_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "stem_step_sched_set": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32]),
    "stem_join_create": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "stem_join_workspace_bytes": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32,
                                                   ctypes.POINTER(ctypes.c_uint64)]),
    "stem_join_contract": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                            ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint32,
                                            ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                            ctypes.c_uint32, ctypes.c_void_p]),
    "stem_join_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "stem_fill_counter": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_int32, ctypes.c_void_p]),
    "stem_xeb_f64": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "stem_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "stem_last_error": (ctypes.c_char_p, []),
}

_lib = None


class StemError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"stemgpu status {status}: {message}")
        self.status = status


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2005_06787_amd.build` "
                "(the HIP path has no fallback)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int) -> None:
    if status != STEM_OK:
        msg = lib().stem_last_error().decode(errors="replace")
        raise StemError(status, msg)
