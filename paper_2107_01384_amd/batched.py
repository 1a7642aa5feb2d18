"""Batched ST-HOSVD binding: many small 3-way float32 blocks in one persistent launch."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import BlockResult, _check, _stream, load, make_opts


class BatchPlan:
    """Owns an atc_batch_plan (block offsets, slots, processing order, launch choice)."""

    def __init__(self, dims, rel_error: float = 1e-3, precision: str = "bf16x3", rule: str = "adaptive",
                 max_sweeps: int = 0, input_offsets=None):
        """input_offsets: element offset of each block in the input arena (None:
        blocks packed back to back in block order)."""
        lib = load()
        dims = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1, 3))
        self.dims = dims
        self.nblocks = int(dims.shape[0])
        self.opts = make_opts(rel_error, precision, None, 1.0, rule, None, max_sweeps, 0)
        offp = None
        if input_offsets is not None:
            self._offsets_in = np.ascontiguousarray(np.asarray(input_offsets, dtype=np.int64).reshape(-1))
            if self._offsets_in.shape[0] != self.nblocks:
                raise ValueError("input_offsets needs one entry per block")
            offp = self._offsets_in.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        h = ctypes.c_void_p()
        _check(lib.atc_batch_plan_create(dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), offp, self.nblocks,
                                         ctypes.byref(self.opts), ctypes.byref(h)))
        self.handle = h
        ie, ce, fe = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        ws = ctypes.c_size_t()
        _check(lib.atc_batch_plan_info(h, ctypes.byref(ie), ctypes.byref(ce), ctypes.byref(fe), ctypes.byref(ws)))
        self.input_elems, self.core_elems, self.factor_elems = ie.value, ce.value, fe.value
        self.workspace_bytes = ws.value
        io = np.zeros(self.nblocks, dtype=np.int64)
        co = np.zeros(self.nblocks, dtype=np.int64)
        fo = np.zeros(self.nblocks, dtype=np.int64)
        p64 = ctypes.POINTER(ctypes.c_int64)
        _check(lib.atc_batch_plan_offsets(h, io.ctypes.data_as(p64), co.ctypes.data_as(p64), fo.ctypes.data_as(p64)))
        self.input_off, self.core_off, self.factor_off = io, co, fo
        self.graph = None

    def allocate(self, device="cuda"):
        """Output arenas, the per-block result records and the workspace."""
        core = torch.empty(max(1, self.core_elems), dtype=torch.float32, device=device)
        fac = torch.empty(max(1, self.factor_elems), dtype=torch.float32, device=device)
        res = torch.zeros(self.nblocks * ctypes.sizeof(BlockResult), dtype=torch.uint8, device=device)
        ws = torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8, device=device)
        return core, fac, res, ws

    def _args(self, arena, core, fac, res, ws):
        return (self.handle, ctypes.c_void_p(arena.data_ptr()), ctypes.c_void_p(core.data_ptr()),
                ctypes.c_void_p(fac.data_ptr()), ctypes.c_void_p(res.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                ws.numel())

    def run(self, arena, core, fac, res, ws, stream=None):
        _check(load().atc_sthosvd_batched(*self._args(arena, core, fac, res, ws), ctypes.c_void_p(_stream(stream))))

    def autotune(self, arena, core, fac, res, ws, reps: int = 5, cache_path: Optional[str] = None, stream=None):
        choice = ctypes.c_int32(-1)
        cp = cache_path.encode() if cache_path else None
        _check(load().atc_batch_autotune(*self._args(arena, core, fac, res, ws), ctypes.c_void_p(_stream(stream)),
                                         reps, cp, ctypes.byref(choice)))
        return choice.value

    def capture(self, arena, core, fac, res, ws, stream=None):
        g = ctypes.c_void_p()
        _check(load().atc_batch_graph_create(*self._args(arena, core, fac, res, ws),
                                             ctypes.c_void_p(_stream(stream)), ctypes.byref(g)))
        if self.graph is not None:
            load().atc_graph_destroy(self.graph)
        self.graph = g
        return g

    def replay(self, stream=None):
        _check(load().atc_graph_launch(self.graph, ctypes.c_void_p(_stream(stream))))

    @staticmethod
    def results(res_tensor) -> np.ndarray:
        """Per-block records as a numpy structured array."""
        dt = np.dtype([("ranks", np.int32, 3), ("status", np.int32), ("norm2", np.float64),
                       ("sse_pred", np.float64), ("tail", np.float64, 3)])
        assert dt.itemsize == ctypes.sizeof(BlockResult)
        return np.frombuffer(res_tensor.cpu().numpy().tobytes(), dtype=dt)

    def core_of(self, core, b: int, ranks):
        n = int(np.prod(ranks))
        return core[self.core_off[b]: self.core_off[b] + n].view(*[int(r) for r in ranks])

    def factor_of(self, fac, b: int, k: int, r: int):
        d = self.dims[b]
        off = int(self.factor_off[b]) + int(sum(int(d[j]) ** 2 for j in range(k)))
        return fac[off: off + int(d[k]) * r].view(int(d[k]), r)

    def __del__(self):
        try:
            lib = load()
            if getattr(self, "graph", None) is not None:
                lib.atc_graph_destroy(self.graph)
            if getattr(self, "handle", None):
                lib.atc_batch_plan_destroy(self.handle)
        except Exception:
            pass


def sthosvd_batched(arena: torch.Tensor, dims, rel_error: float = 1e-3, precision: str = "bf16x3"):
    """One-shot convenience: plan, allocate, run; returns (plan, core, factors, results)."""
    plan = BatchPlan(dims, rel_error, precision)
    core, fac, res, ws = plan.allocate(arena.device)
    plan.run(arena, core, fac, res, ws)
    return plan, core, fac, res
