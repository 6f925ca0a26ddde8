"""Python face of libstemgpu: a plan object over the C-ABI.

A *stem network* is plain data (the same dictionary layout the planner
writes):

    {"open_labels": [...], "sliced_labels": [...], "proj_labels": [...],
     "stem": {"labels": [...], "data": complex array (2,)*rank},
     "branches": [{"labels": [...], "data": complex array}, ...]}

This module only marshals arguments: host arrays become C pointers, device
memory and streams come from PyTorch, and every step of the contraction runs
in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _capi as C


def _i32(values) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(list(values), dtype=np.int32))


def _c64(arr) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(arr, dtype=np.complex64).reshape(-1))


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class _Desc:
    """stem_plan_desc plus the host arrays it points into (kept alive)."""

    def __init__(self, net: dict, precision: str = "fp32", stem_device_ptr: int | None = None,
                 max_rank: int = 0, shapes_only: bool = False):
        if precision not in C.PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(C.PRECISIONS)}")
        self.open = _i32(net.get("open_labels", []))
        self.sliced = _i32(net.get("sliced_labels", []))
        self.proj = _i32(net.get("proj_labels", []))
        self.stem_labels = _i32(net["stem"]["labels"])
        branches = net.get("branches", [])
        self.ranks = _i32(len(b["labels"]) for b in branches)
        self.blabels = _i32(x for b in branches for x in b["labels"])
        if not len(self.blabels):
            self.blabels = np.zeros(1, dtype=np.int32)
        if shapes_only:
            # stem_plan_validate / stem_plan_steps read labels only; the data
            # pointers must just be non-null
            self.bdata = np.zeros(1, dtype=np.complex64)
        else:
            self.bdata = (np.concatenate([_c64(b["data"]) for b in branches])
                          if branches else np.zeros(1, dtype=np.complex64))
        d = C.stem_plan_desc()
        d.n_open, d.open_labels = len(self.open), _ptr(self.open, ctypes.c_int32)
        d.n_sliced, d.sliced_labels = len(self.sliced), _ptr(self.sliced, ctypes.c_int32)
        d.n_proj, d.proj_labels = len(self.proj), _ptr(self.proj, ctypes.c_int32)
        d.stem_rank, d.stem_labels = len(self.stem_labels), _ptr(self.stem_labels, ctypes.c_int32)
        if stem_device_ptr is not None:
            d.stem_data = ctypes.c_void_p(int(stem_device_ptr))
            d.stem_on_device = 1
        elif shapes_only:
            self.stem = np.zeros(1, dtype=np.complex64)
            d.stem_data = ctypes.c_void_p(self.stem.ctypes.data)
            d.stem_on_device = 0
        else:
            self.stem = _c64(net["stem"]["data"])
            if self.stem.size != 1 << len(self.stem_labels):
                raise ValueError("stem data size does not match its rank")
            d.stem_data = ctypes.c_void_p(self.stem.ctypes.data)
            d.stem_on_device = 0
        d.n_branches = len(branches)
        d.branch_ranks = _ptr(self.ranks, ctypes.c_int32)
        d.branch_labels = _ptr(self.blabels, ctypes.c_int32)
        d.branch_data = ctypes.c_void_p(self.bdata.ctypes.data)
        d.precision = C.PRECISIONS[precision]
        d.max_rank = int(max_rank)
        self.desc = d


def stem_plan_validate(net: dict, precision: str = "fp32", max_rank: int = 0) -> dict:
    """Host-only check of a stem network (labels only; data may be absent);
    returns the plan summary."""
    d = _Desc(net, precision, max_rank=max_rank, shapes_only=True)
    s = C.stem_plan_summary()
    C.check(C.lib().stem_plan_validate(ctypes.byref(d.desc), ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in s._fields_}


class Plan:
    """A plan living on the current GPU (paper §A.2: stem order, branches,
    sliced set).  ``contract`` sums slices into FP64 amplitudes."""

    def __init__(self, net: dict, precision: str = "fp32", stream=None,
                 stem_device=None, max_rank: int = 0):
        import torch  # device memory and streams only

        self._torch = torch
        ptr = None
        if stem_device is not None:
            if not (stem_device.is_cuda and stem_device.dtype == torch.complex64
                    and stem_device.is_contiguous()):
                raise ValueError("stem_device must be a contiguous complex64 CUDA tensor")
            ptr = stem_device.data_ptr()
        self._d = _Desc(net, precision, ptr, max_rank)
        self.precision = precision
        self.n_open = len(self._d.open)
        self.n_sliced = len(self._d.sliced)
        self.n_proj = len(self._d.proj)
        h = ctypes.c_void_p()
        C.check(C.lib().stem_plan_create(ctypes.byref(self._d.desc), _stream_handle(stream),
                                         ctypes.byref(h)))
        self._h = h
        self._ws = None
        # host copies are no longer needed
        self._d.bdata = None
        self._d.stem = None

    # -- info -------------------------------------------------------------
    def summary(self) -> dict:
        s = C.stem_plan_summary()
        C.check(C.lib().stem_plan_summary_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def workspace_bytes(self, slices_in_flight: int = 1) -> int:
        b = ctypes.c_uint64()
        C.check(C.lib().stem_plan_workspace_bytes(self._h, int(slices_in_flight),
                                                  ctypes.byref(b)))
        return int(b.value)

    def default_slices_in_flight(self, n_slices: int) -> int:
        """Slices per launch: all of them, up to 256 and a 16 GiB workspace."""
        per = max(1, self.workspace_bytes(1))
        return int(max(1, min(n_slices, 256, (16 << 30) // per)))

    def step_info(self, i: int) -> dict:
        s = C.stem_step_info()
        C.check(C.lib().stem_step_info_get(self._h, int(i), ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def steps(self) -> list[dict]:
        return [self.step_info(i) for i in range(self.summary()["n_steps"])]

    def set_schedule(self, step: int, tm: int = 1, ntw: int = 1, blocks: int = 4096,
                     lds: int = -1, algo: int = 0) -> dict:
        """Set one step's launch schedule (C-ABI stem_step_sched_set); returns
        the step info with the schedule as the kernels will run it."""
        C.check(C.lib().stem_step_sched_set(self._h, int(step), int(tm), int(ntw), int(blocks),
                                            int(lds), int(algo)))
        return self.step_info(step)

    # -- work -------------------------------------------------------------
    def workspace(self, slices_in_flight: int = 1):
        """Device workspace (cached on the plan) for that many slices per launch."""
        torch = self._torch
        need = self.workspace_bytes(slices_in_flight)
        if self._ws is None or self._ws.numel() != need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        return self._ws

    def contract(self, s0: int = 0, s1: int | None = None, proj=None, out=None,
                 accumulate: bool = False, time_steps: bool = False, stream=None,
                 slices_in_flight: int | None = None):
        """Sum of slices [s0, s1) for each projected assignment in ``proj``.

        Returns (or fills) a complex128 CUDA tensor [n_batch, 2^n_open].
        ``slices_in_flight`` slices run per kernel launch (default: all of
        the range, within the limits of ``default_slices_in_flight``).
        """
        torch = self._torch
        if s1 is None:
            s1 = 1 << self.n_sliced
        if slices_in_flight is None:
            slices_in_flight = self.default_slices_in_flight(max(1, s1 - s0))
        if proj is None:
            proj = [0]
        proj_arr = np.ascontiguousarray(np.asarray(list(proj), dtype=np.uint64))
        nb = len(proj_arr)
        if out is None:
            out = torch.empty((nb, 1 << self.n_open), dtype=torch.complex128, device="cuda")
        if not (out.is_cuda and out.dtype == torch.complex128 and out.is_contiguous()
                and out.numel() == nb << self.n_open):
            raise ValueError("out must be a contiguous complex128 CUDA tensor [n_batch, 2^n_open]")
        ws = self.workspace(slices_in_flight)
        flags = (C.STEM_ACCUMULATE if accumulate else 0) | (C.STEM_TIME_STEPS if time_steps else 0)
        C.check(C.lib().stem_contract(
            self._h, int(s0), int(s1), _ptr(proj_arr, ctypes.c_uint64), nb,
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(out.data_ptr()),
            flags, _stream_handle(stream)))
        return out

    def tune(self, slices_in_flight: int | None = None, reps: int = 3,
             cache_path: str | None = None, stream=None) -> list[dict]:
        """Autotune every step's product schedule (C-ABI stem_tune) at the
        given slices per launch; returns the step infos after tuning."""
        if slices_in_flight is None:
            slices_in_flight = self.default_slices_in_flight(1 << self.n_sliced)
        ws = self.workspace(slices_in_flight)
        path = cache_path.encode() if cache_path else None
        C.check(C.lib().stem_tune(self._h, int(slices_in_flight), ctypes.c_void_p(ws.data_ptr()),
                                  ws.numel(), int(reps), path, _stream_handle(stream)))
        return self.steps()

    def close(self):
        if getattr(self, "_h", None):
            C.lib().stem_plan_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Join:
    """Two plans joined at the root (C-ABI stem_join_*, paper §A.2): per
    slice, the two final stems are contracted over the labels open in both;
    ``open_labels`` (the labels open in exactly one plan) orders the result."""

    def __init__(self, left: Plan, right: Plan, open_labels):
        self.left, self.right = left, right
        self.open = [int(x) for x in open_labels]
        self.n_open = len(self.open)
        self.n_sliced = left.n_sliced
        arr = _i32(self.open)
        h = ctypes.c_void_p()
        C.check(C.lib().stem_join_create(left._h, right._h, self.n_open,
                                         _ptr(arr, ctypes.c_int32), ctypes.byref(h)))
        self._h = h
        self._ws = None

    def workspace_bytes(self, slices_in_flight: int = 1) -> int:
        b = ctypes.c_uint64()
        C.check(C.lib().stem_join_workspace_bytes(self._h, int(slices_in_flight),
                                                  ctypes.byref(b)))
        return int(b.value)

    def contract(self, s0: int = 0, s1: int | None = None, proj=None, out=None,
                 accumulate: bool = False, stream=None, slices_in_flight: int | None = None):
        """Sum over slices [s0, s1) of the joined value, per projected
        assignment: a complex128 CUDA tensor [n_batch, 2^n_open]."""
        import torch

        if s1 is None:
            s1 = 1 << self.n_sliced
        if slices_in_flight is None:
            per = max(1, self.workspace_bytes(1))
            slices_in_flight = int(max(1, min(max(1, s1 - s0), 256, (16 << 30) // per)))
        proj_arr = np.ascontiguousarray(np.asarray(list(proj if proj is not None else [0]),
                                                   dtype=np.uint64))
        nb = len(proj_arr)
        if out is None:
            out = torch.empty((nb, 1 << self.n_open), dtype=torch.complex128, device="cuda")
        if not (out.is_cuda and out.dtype == torch.complex128 and out.is_contiguous()
                and out.numel() == nb << self.n_open):
            raise ValueError("out must be a contiguous complex128 CUDA tensor [n_batch, 2^n_open]")
        need = self.workspace_bytes(slices_in_flight)
        if self._ws is None or self._ws.numel() != need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        C.check(C.lib().stem_join_contract(
            self._h, int(s0), int(s1), _ptr(proj_arr, ctypes.c_uint64), nb,
            ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(),
            ctypes.c_void_p(out.data_ptr()), C.STEM_ACCUMULATE if accumulate else 0,
            _stream_handle(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            C.lib().stem_join_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Slice ranges of several plans recorded as one HIP graph (C-ABI
    stem_batch_*).  ``launch()`` replays it: every plan's output is
    recomputed (or added to, with ``accumulate``)."""

    def __init__(self, plans, ranges, proj=None, outs=None, ws_bytes: int | None = None,
                 accumulate: bool = False, stream=None):
        import torch

        n = len(plans)
        if len(ranges) != n:
            raise ValueError("one (s0, s1) range per plan")
        self.plans = list(plans)
        self.outs = outs if outs is not None else [
            torch.empty(1 << p.n_open, dtype=torch.complex128, device="cuda") for p in plans]
        if ws_bytes is None:
            ws_bytes = 0
            for p, (a, b) in zip(plans, ranges):
                ws_bytes = max(ws_bytes, p.workspace_bytes(p.default_slices_in_flight(max(1, b - a))))
            ws_bytes *= n
        self.ws = torch.empty(max(256, int(ws_bytes)), dtype=torch.uint8, device="cuda")
        hp = (ctypes.c_void_p * n)(*[p._h for p in plans])
        a0 = (ctypes.c_uint64 * n)(*[int(r[0]) for r in ranges])
        a1 = (ctypes.c_uint64 * n)(*[int(r[1]) for r in ranges])
        pr = (ctypes.c_uint64 * n)(*([int(x) for x in proj] if proj is not None else [0] * n))
        op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in self.outs])
        h = ctypes.c_void_p()
        C.check(C.lib().stem_batch_create(
            n, hp, a0, a1, pr, op, ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
            C.STEM_ACCUMULATE if accumulate else 0, _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        C.check(C.lib().stem_batch_launch(self._h, _stream_handle(stream)))
        return self.outs

    def close(self):
        if getattr(self, "_h", None):
            C.lib().stem_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stem_fill_counter(dst, seed: int, scale_log2: int, stream=None) -> None:
    """Fill a complex64 CUDA tensor with the counter-based test tensor."""
    C.check(C.lib().stem_fill_counter(ctypes.c_void_p(dst.data_ptr()), dst.numel(), int(seed),
                                      int(scale_log2), _stream_handle(stream)))


def stem_xeb_f64(amps, n_qubits: int, out=None, stream=None):
    """(XEB, sum |a|^2) of a complex128 CUDA tensor of amplitudes, in FP64."""
    import torch

    if out is None:
        out = torch.empty(2, dtype=torch.float64, device="cuda")
    C.check(C.lib().stem_xeb_f64(ctypes.c_void_p(amps.data_ptr()), amps.numel(), int(n_qubits),
                                 ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out
