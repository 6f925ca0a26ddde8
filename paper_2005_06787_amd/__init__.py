"""Sliced-stem tensor-network contraction on MI355X (gfx950).

The hot path of arXiv 2005.06787 (paper §A.1-§A.3): a stem tensor absorbs
pre-computed branch tensors step by step, repeated for every assignment of
the sliced labels, and the slices are summed in FP64.  The work runs in the
HIP kernels of ``_lib/libstemgpu.so`` behind the C-ABI of
``include/stemgpu.h``; this package marshals arguments and plans networks.
"""

from .stem import Batch, Join, Plan, stem_fill_counter, stem_plan_validate, stem_xeb_f64  # noqa: F401
