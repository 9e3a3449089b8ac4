"""Batched transforms of uneven sizes: a torch-facing wrapper of the plan ABI.

    plan = Plan2D(inputs, outputs, levels, inverse=False)   # lists of tensors
    plan.execute()                                          # one persistent launch

All tensors live on the same GPU with one storage dtype; the plan keeps them
alive.  The workspace is a torch byte tensor; the plan is uploaded on the
current stream at construction (and after ``tune()``).  ``execute()`` may be
captured into a CUDA/HIP graph and replayed.
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi
from .transform import DTYPE_CODES


class _Plan:
    def __init__(self, items, count, dtype, inverse, create, tensors):
        self._tensors = tensors
        self._ptr = ctypes.c_void_p()
        _abi.check(create(items, count, DTYPE_CODES[dtype], int(inverse), ctypes.byref(self._ptr)))
        nbytes = ctypes.c_size_t()
        _abi.check(_abi.haar_plan_workspace_size(self._ptr, ctypes.byref(nbytes)))
        self.workspace = torch.empty(max(256, nbytes.value), dtype=torch.uint8,
                                     device=tensors[0].device)
        self.upload()

    def _stream(self):
        return torch.cuda.current_stream(self.workspace.device).cuda_stream

    def upload(self):
        _abi.check(_abi.haar_plan_upload(self._ptr, self.workspace.data_ptr(), self._stream()))

    def execute(self):
        _abi.check(_abi.haar_plan_execute(self._ptr, self.workspace.data_ptr(), self._stream()))

    def tune(self) -> int:
        """Time the plan's configurations (overwrites the outputs) and keep the fastest."""
        choice = ctypes.c_int32(-1)
        _abi.check(_abi.haar_plan_tune(self._ptr, self.workspace.data_ptr(), self._stream(),
                                       ctypes.byref(choice)))
        return choice.value

    def set_config(self, config: int):
        _abi.check(_abi.haar_plan_set_config(self._ptr, int(config)))
        self.upload()

    def info(self):
        tiles, grid = ctypes.c_int64(), ctypes.c_int32()
        _abi.check(_abi.haar_plan_info(self._ptr, ctypes.byref(tiles), ctypes.byref(grid)))
        return tiles.value, grid.value

    def __del__(self):
        ptr = getattr(self, "_ptr", None)
        if ptr is not None and ptr.value:
            torch.cuda.synchronize(self.workspace.device)
            _abi.haar_plan_destroy(ptr)
            self._ptr = None


def _check_tensors(inputs, outputs):
    if len(inputs) != len(outputs) or not inputs:
        raise ValueError("need the same non-zero number of inputs and outputs")
    dt = inputs[0].dtype
    for a, b in zip(inputs, outputs):
        if a.dtype != dt or b.dtype != dt or not a.is_cuda or not b.is_cuda:
            raise ValueError("all tensors must be GPU tensors of one dtype")
        if not a.is_contiguous() or not b.is_contiguous() or a.shape != b.shape:
            raise ValueError("inputs/outputs must be contiguous and pairwise of equal shape")
    return dt


class Plan2D(_Plan):
    """Plan over [h_i, w_i] images; levels: int or list (1..5)."""

    def __init__(self, inputs, outputs, levels, inverse=False):
        dt = _check_tensors(inputs, outputs)
        lv = levels if isinstance(levels, (list, tuple)) else [levels] * len(inputs)
        items = (_abi.Item2D * len(inputs))()
        for i, (a, b) in enumerate(zip(inputs, outputs)):
            items[i] = _abi.Item2D(a.data_ptr(), b.data_ptr(), a.shape[-2], a.shape[-1], int(lv[i]))
        super().__init__(items, len(inputs), dt, inverse, _abi.haar_plan_create_2d,
                         list(inputs) + list(outputs))


class Plan1D(_Plan):
    """Plan over [n_i] signals; levels: int or list."""

    def __init__(self, inputs, outputs, levels, inverse=False):
        dt = _check_tensors(inputs, outputs)
        lv = levels if isinstance(levels, (list, tuple)) else [levels] * len(inputs)
        items = (_abi.Item1D * len(inputs))()
        for i, (a, b) in enumerate(zip(inputs, outputs)):
            items[i] = _abi.Item1D(a.data_ptr(), b.data_ptr(), a.shape[-1], int(lv[i]))
        super().__init__(items, len(inputs), dt, inverse, _abi.haar_plan_create_1d,
                         list(inputs) + list(outputs))
