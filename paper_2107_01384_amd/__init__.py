"""Python binding of libatc, the MI355X (gfx950) ST-HOSVD library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libatc.so`` behind the C ABI declared in ``include/atc.h``.
PyTorch provides device memory and the current HIP stream.  There is no CPU
fallback: if the library is missing or no GPU is present the calls raise.

Entry points (same names as the C ABI, minus the ``atc_`` prefix):
  * ``sthosvd(x, rel_error, ...)``            -- ST-HOSVD (Algorithm 1, Section 3.2)
  * ``BatchPlan`` / ``sthosvd_batched(...)``  -- many small blocks, one persistent launch
  * ``reconstruct(core, factors)``            -- Tucker reconstruction (Section 3.2)
  * ``reconstruct_backward(core, factors, dxhat)`` and ``TuckerReconstruct``
    (a ``torch.autograd.Function`` whose backward is the hand-written adjoint).
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libatc.so")
MAX_DIMS = 8

ATC_F32, ATC_F64 = 0, 1
PRECISIONS = {"native": 0, "bf16x3": 1, "f64acc": 2}
_PREC_NAMES = {v: k for k, v in PRECISIONS.items()}
RULES = {"adaptive": 0, "equal": 1}
STATUS = {
    0: "ok", -1: "invalid argument", -2: "unsupported", -3: "workspace too small", -4: "device error",
    -5: "eigensolver did not converge", -6: "non-finite input", -7: "internal error",
}


class AtcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("atc status %d (%s): %s" % (status, STATUS.get(status, "?"), message))
        self.status = status


class Shape(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32), ("dims", ctypes.c_int64 * MAX_DIMS)]


class Opts(ctypes.Structure):
    _fields_ = [
        ("rel_error", ctypes.c_double), ("rtmss", ctypes.c_double), ("precision", ctypes.c_int32),
        ("rank_rule", ctypes.c_int32), ("has_order", ctypes.c_int32), ("mode_order", ctypes.c_int32 * MAX_DIMS),
        ("has_fixed_ranks", ctypes.c_int32), ("fixed_ranks", ctypes.c_int32 * MAX_DIMS),
        ("max_sweeps", ctypes.c_int32), ("eig_path", ctypes.c_int32), ("profile", ctypes.c_int32),
        ("no_precision_guard", ctypes.c_int32), ("no_host_wait", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("ranks", ctypes.c_int64 * MAX_DIMS), ("order", ctypes.c_int32 * MAX_DIMS), ("norm2", ctypes.c_double),
        ("sse_pred", ctypes.c_double), ("tail", ctypes.c_double * MAX_DIMS), ("budget", ctypes.c_double * MAX_DIMS),
        ("eig_path", ctypes.c_int32 * MAX_DIMS), ("eig_sweeps", ctypes.c_int32 * MAX_DIMS),
        ("elapsed_ms", ctypes.c_double), ("gram_ms", ctypes.c_double * MAX_DIMS),
        ("reduce_ms", ctypes.c_double * MAX_DIMS), ("eig_ms", ctypes.c_double * MAX_DIMS),
        ("ttm_ms", ctypes.c_double * MAX_DIMS), ("gram_prec", ctypes.c_int32 * MAX_DIMS),
    ]


class BlockResult(ctypes.Structure):
    _fields_ = [
        ("ranks", ctypes.c_int32 * 3), ("status", ctypes.c_int32), ("norm2", ctypes.c_double),
        ("sse_pred", ctypes.c_double), ("tail", ctypes.c_double * 3),
    ]


class QuantInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("k", ctypes.c_int32), ("plane", ctypes.c_int32), ("block_len", ctypes.c_int32),
        ("n", ctypes.c_int64), ("count", ctypes.c_int64), ("nblocks", ctypes.c_int64), ("words", ctypes.c_int64),
        ("sse", ctypes.c_double), ("pad", ctypes.c_int64),
    ]


QUANT_KZERO = -(2 ** 31)


class HybridOut(ctypes.Structure):
    _fields_ = [
        ("core_enc", ctypes.c_void_p), ("core_info", ctypes.c_void_p), ("core_q", ctypes.c_void_p),
        ("sigma2", ctypes.c_void_p), ("signs", ctypes.c_void_p),
        ("factor_signed", ctypes.c_void_p * MAX_DIMS), ("factor_coef", ctypes.c_void_p * MAX_DIMS),
        ("factor_enc", ctypes.c_void_p * MAX_DIMS), ("factor_info", ctypes.c_void_p * MAX_DIMS),
        ("factor_q", ctypes.c_void_p * MAX_DIMS), ("factor_term", ctypes.c_void_p), ("status", ctypes.c_void_p),
    ]

# (name, restype, argtypes) of every symbol include/atc.h declares
_VP, _SZ, _I64, _I32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int32
_P = ctypes.POINTER
SIGNATURES = [
    ("atc_default_opts", None, [_P(Opts)]),
    ("atc_sthosvd_workspace_size", _SZ, [_P(Shape), _P(Opts)]),
    ("atc_sthosvd", _I32, [_VP, _P(Shape), _P(Opts), _VP, _P(_VP), _P(Result), _VP, _SZ, _VP]),
    ("atc_sthosvd_finish", _I32, [_P(Shape), _P(Opts), _VP, _SZ, _P(Result), _VP]),
    ("atc_batch_plan_create", _I32, [_P(_I32), _P(_I64), _I64, _P(Opts), _P(_VP)]),
    ("atc_batch_plan_destroy", None, [_VP]),
    ("atc_batch_plan_info", _I32, [_VP, _P(_I64), _P(_I64), _P(_I64), _P(_SZ)]),
    ("atc_batch_plan_offsets", _I32, [_VP, _P(_I64), _P(_I64), _P(_I64)]),
    ("atc_sthosvd_batched", _I32, [_VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    ("atc_batch_autotune", _I32, [_VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP, _I32, ctypes.c_char_p, _P(_I32)]),
    ("atc_batch_graph_create", _I32, [_VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP, _P(_VP)]),
    ("atc_graph_launch", _I32, [_VP, _VP]),
    ("atc_graph_destroy", None, [_VP]),
    ("atc_reconstruct_workspace_size", _SZ, [_P(Shape), _P(_I64)]),
    ("atc_reconstruct", _I32, [_P(Shape), _P(_I64), _VP, _P(_VP), _VP, _VP, _SZ, _VP]),
    ("atc_reconstruct_noalloc", _I32, [_P(Shape), _P(_I64), _VP, _P(_VP), _VP, _VP]),
    ("atc_reconstruct_backward_workspace_size", _SZ, [_P(Shape), _P(_I64)]),
    ("atc_reconstruct_backward", _I32, [_P(Shape), _P(_I64), _VP, _P(_VP), _VP, _VP, _P(_VP), _VP, _SZ, _VP]),
    ("atc_quantize_max_words", _SZ, [_I64, _I32]),
    ("atc_quantize_workspace_size", _SZ, [_I64, _I32]),
    ("atc_quantize_core", _I32, [_VP, _I32, _I64, ctypes.c_double, _I32, _VP, _SZ, _VP, _VP, _SZ, _VP]),
    ("atc_dequantize_workspace_size", _SZ, [_I64, _I32]),
    ("atc_dequantize_core", _I32, [_VP, _I64, _I32, _I32, _VP, _VP, _VP, _SZ, _VP]),
    ("atc_householder_workspace_size", _SZ, [_I64, _I64]),
    ("atc_factor_householder", _I32, [_VP, _I32, _I64, _I64, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    ("atc_factor_weight_coefficients", _I32, [_VP, _VP, _I64, _I64, _VP]),
    ("atc_factor_from_householder", _I32, [_VP, _VP, _I64, _I64, _I32, _VP, _VP, _SZ, _VP]),
    ("atc_core_slice_norms_count", _SZ, [_P(Shape)]),
    ("atc_core_slice_norms", _I32, [_VP, _P(Shape), _VP, _VP]),
    ("atc_core_apply_signs", _I32, [_VP, _P(Shape), _VP, _VP]),
    ("atc_factor_error_term", _I32, [_VP, _VP, _I32, _I64, _I64, _VP, _VP, _VP]),
    ("atc_hybrid_workspace_size", _SZ, [_P(Shape), _P(_I64), _I32]),
    ("atc_hybrid_quantize", _I32, [_VP, _P(Shape), _P(_VP), _P(_I64), ctypes.c_double, ctypes.c_double, _I32,
                                   _P(HybridOut), _VP, _SZ, _VP]),
    ("atc_status_string", ctypes.c_char_p, [_I32]),
    ("atc_last_error", ctypes.c_char_p, []),
    ("atc_version", ctypes.c_char_p, []),
    ("atc_finalize", None, []),
]

_lib = None


def load(path: str = LIB_PATH):
    """Loads libatc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libatc.so is not built (%s); run paper_2107_01384_amd.build.build()" % path)
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    atexit.register(_finalize)
    return lib


def _finalize():
    """At interpreter exit, before the HIP runtime shuts down: wait for the
    device, then release the pinned report block and events of this thread."""
    if _lib is None:
        return
    try:
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    finally:
        _lib.atc_finalize()


def _check(status: int):
    if status != 0:
        raise AtcError(status, load().atc_last_error().decode(errors="replace"))


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _require_gpu(t: torch.Tensor, what: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.dtype not in (torch.float32, torch.float64):
        raise ValueError("%s must be float32 or float64" % what)


def _shape(dims: Sequence[int], dtype: torch.dtype) -> Shape:
    s = Shape()
    s.ndim = len(dims)
    s.dtype = ATC_F64 if dtype == torch.float64 else ATC_F32
    for i, n in enumerate(dims):
        s.dims[i] = int(n)
    return s


def make_opts(rel_error: float = 1e-3, precision: str = "native", order=None, rtmss: float = 1.0,
              rule: str = "adaptive", fixed_ranks=None, max_sweeps: int = 0, eig_path: int = 0,
              profile: bool = False, precision_guard: bool = True, no_host_wait: bool = False) -> Opts:
    o = Opts()
    load().atc_default_opts(ctypes.byref(o))
    o.rel_error = float(rel_error)
    o.rtmss = float(rtmss)
    o.precision = PRECISIONS[precision]
    o.rank_rule = RULES[rule]
    if order is not None:
        o.has_order = 1
        for i, k in enumerate(order):
            o.mode_order[i] = int(k)
    if fixed_ranks is not None:
        o.has_fixed_ranks = 1
        for i, r in enumerate(fixed_ranks):
            o.fixed_ranks[i] = int(r)
    o.max_sweeps = int(max_sweeps)
    o.eig_path = int(eig_path)
    o.profile = 1 if profile else 0
    o.no_precision_guard = 0 if precision_guard else 1
    o.no_host_wait = 1 if no_host_wait else 0
    return o


@dataclass
class Tucker:
    core: torch.Tensor
    factors: List[torch.Tensor]
    ranks: List[int]
    order: List[int]
    norm2: float
    sse_pred: float
    tails: List[float]
    budgets: List[float]
    eig_path: List[int]
    eig_sweeps: List[int]
    elapsed_ms: float
    phase_ms: dict
    gram_prec: List[str]


def sthosvd_workspace_size(dims, dtype=torch.float32, **opt_kw) -> int:
    s = _shape(dims, dtype)
    o = make_opts(**opt_kw)
    n = load().atc_sthosvd_workspace_size(ctypes.byref(s), ctypes.byref(o))
    if n == 0:
        _check(-1)
    return int(n)


def sthosvd(x: torch.Tensor, rel_error: float = 1e-3, precision: str = "native", order=None, rtmss: float = 1.0,
            rule: str = "adaptive", fixed_ranks=None, max_sweeps: int = 0, eig_path: int = 0,
            workspace: Optional[torch.Tensor] = None, stream=None, profile: bool = False,
            out: Optional[tuple] = None, precision_guard: bool = True, no_host_wait: bool = False) -> Tucker:
    """ST-HOSVD of x (GPU tensor) to relative error rel_error; see atc_sthosvd in include/atc.h.
    The ranks and figures of the result are final on return; core and factors
    are written in the order of `stream` (torch's current stream by default).
    With no_host_wait (fixed_ranks required) nothing waits for the device, so
    the call can be captured in a graph: norm2, sse_pred, tails, budgets and
    eig_sweeps are then zero until sthosvd_finish reads them."""
    lib = load()
    _require_gpu(x, "x")
    dims = list(x.shape)
    s = _shape(dims, x.dtype)
    o = make_opts(rel_error, precision, order, rtmss, rule, fixed_ranks, max_sweeps, eig_path, profile,
                  precision_guard, no_host_wait)
    need = lib.atc_sthosvd_workspace_size(ctypes.byref(s), ctypes.byref(o))
    if need == 0:
        _check(-1)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    if out is not None:  # preallocated (core, [factors]) buffers of full capacity
        core, facs = out
    else:
        core = torch.empty(x.numel(), dtype=x.dtype, device=x.device)
        facs = [torch.empty(n * n, dtype=x.dtype, device=x.device) for n in dims]
    fptr = (ctypes.c_void_p * len(dims))(*[f.data_ptr() for f in facs])
    res = Result()
    st = lib.atc_sthosvd(ctypes.c_void_p(x.data_ptr()), ctypes.byref(s), ctypes.byref(o),
                         ctypes.c_void_p(core.data_ptr()), fptr, ctypes.byref(res),
                         ctypes.c_void_p(workspace.data_ptr()), need, ctypes.c_void_p(_stream(stream)))
    _check(st)
    d = len(dims)
    ranks = [int(res.ranks[k]) for k in range(d)]
    ncore = 1
    for r in ranks:
        ncore *= r
    return Tucker(
        core=core[:ncore].view(*ranks),
        factors=[facs[k][: dims[k] * ranks[k]].view(dims[k], ranks[k]) for k in range(d)],
        ranks=ranks, order=[int(res.order[k]) for k in range(d)], norm2=float(res.norm2),
        sse_pred=float(res.sse_pred), tails=[float(res.tail[k]) for k in range(d)],
        budgets=[float(res.budget[k]) for k in range(d)], eig_path=[int(res.eig_path[k]) for k in range(d)],
        eig_sweeps=[int(res.eig_sweeps[k]) for k in range(d)], elapsed_ms=float(res.elapsed_ms),
        phase_ms={name: [float(getattr(res, name + "_ms")[k]) for k in range(d)]
                  for name in ("gram", "reduce", "eig", "ttm")},
        gram_prec=[_PREC_NAMES[int(res.gram_prec[k])] for k in range(d)])


def sthosvd_finish(dims, dtype, workspace: torch.Tensor, stream=None, **opt_kw) -> dict:
    """Waits for `stream` after a no_host_wait call (or a graph replay of one)
    made with `workspace` and the same options, and returns the figures that
    call left on the device; raises on the status it recorded.  See
    atc_sthosvd_finish."""
    lib = load()
    if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda:
        raise ValueError("workspace must be a GPU tensor")
    d = len(dims)
    s = _shape(dims, dtype)
    o = make_opts(**opt_kw, no_host_wait=True)
    res = Result()
    _check(lib.atc_sthosvd_finish(ctypes.byref(s), ctypes.byref(o), ctypes.c_void_p(workspace.data_ptr()),
                                  workspace.numel() * workspace.element_size(), ctypes.byref(res),
                                  ctypes.c_void_p(_stream(stream))))
    return dict(norm2=float(res.norm2), sse_pred=float(res.sse_pred), tails=[float(res.tail[k]) for k in range(d)],
                budgets=[float(res.budget[k]) for k in range(d)],
                eig_sweeps=[int(res.eig_sweeps[k]) for k in range(d)])


# ----------------------------------------------------------------- reconstruction
def _ranks_arr(ranks):
    a = (ctypes.c_int64 * MAX_DIMS)()
    for i, r in enumerate(ranks):
        a[i] = int(r)
    return a


def reconstruct(core: torch.Tensor, factors: Sequence[torch.Tensor], stream=None) -> torch.Tensor:
    """X~ = (U_0, ..., U_{d-1}) . G; see atc_reconstruct."""
    lib = load()
    _require_gpu(core, "core")
    for f in factors:
        _require_gpu(f, "factor")
        if f.dtype != core.dtype:
            raise ValueError("factors must have the core's dtype")
    dims = [int(f.shape[0]) for f in factors]
    ranks = [int(f.shape[1]) for f in factors]
    if list(core.shape) != ranks:
        raise ValueError("core shape %s does not match factor ranks %s" % (list(core.shape), ranks))
    s = _shape(dims, core.dtype)
    ra = _ranks_arr(ranks)
    need = lib.atc_reconstruct_workspace_size(ctypes.byref(s), ra)
    if need == 0:
        _check(-1)
    ws = torch.empty(need, dtype=torch.uint8, device=core.device)
    out = torch.empty(dims, dtype=core.dtype, device=core.device)
    fptr = (ctypes.c_void_p * len(dims))(*[f.data_ptr() for f in factors])
    _check(lib.atc_reconstruct(ctypes.byref(s), ra, ctypes.c_void_p(core.data_ptr()), fptr,
                               ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), need,
                               ctypes.c_void_p(_stream(stream))))
    return out


def reconstruct_noalloc(core: torch.Tensor, factors: Sequence[torch.Tensor], out: torch.Tensor,
                        stream=None) -> torch.Tensor:
    """X~ = (U_0, ..., U_{d-1}) . G into the caller's `out`; see
    atc_reconstruct_noalloc (intermediates in the library's device scratch)."""
    lib = load()
    _require_gpu(core, "core")
    _require_gpu(out, "out")
    for f in factors:
        _require_gpu(f, "factor")
        if f.dtype != core.dtype:
            raise ValueError("factors must have the core's dtype")
    dims = [int(f.shape[0]) for f in factors]
    ranks = [int(f.shape[1]) for f in factors]
    if list(core.shape) != ranks:
        raise ValueError("core shape %s does not match factor ranks %s" % (list(core.shape), ranks))
    if list(out.shape) != dims or out.dtype != core.dtype:
        raise ValueError("out must be a %s tensor of shape %s" % (core.dtype, dims))
    s = _shape(dims, core.dtype)
    fptr = (ctypes.c_void_p * len(dims))(*[f.data_ptr() for f in factors])
    _check(lib.atc_reconstruct_noalloc(ctypes.byref(s), _ranks_arr(ranks), ctypes.c_void_p(core.data_ptr()), fptr,
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream(stream))))
    return out


def reconstruct_backward(core: torch.Tensor, factors: Sequence[torch.Tensor], dxhat: torch.Tensor,
                         need_core: bool = True, need_factors=None, stream=None):
    """(dL/dG, [dL/dU_n]) for R = dL/dX~ = dxhat; see atc_reconstruct_backward."""
    lib = load()
    _require_gpu(core, "core")
    _require_gpu(dxhat, "dxhat")
    dims = [int(f.shape[0]) for f in factors]
    ranks = [int(f.shape[1]) for f in factors]
    if list(dxhat.shape) != dims:
        raise ValueError("dxhat shape must equal the full tensor shape")
    d = len(dims)
    if need_factors is None:
        need_factors = [True] * d
    s = _shape(dims, core.dtype)
    ra = _ranks_arr(ranks)
    need = lib.atc_reconstruct_backward_workspace_size(ctypes.byref(s), ra)
    if need == 0:
        _check(-1)
    ws = torch.empty(need, dtype=torch.uint8, device=core.device)
    dcore = torch.empty_like(core) if need_core else None
    dfs = [torch.empty(dims[k], ranks[k], dtype=core.dtype, device=core.device) if need_factors[k] else None
           for k in range(d)]
    fptr = (ctypes.c_void_p * d)(*[f.data_ptr() for f in factors])
    dptr = (ctypes.c_void_p * d)(*[(t.data_ptr() if t is not None else None) for t in dfs])
    _check(lib.atc_reconstruct_backward(ctypes.byref(s), ra, ctypes.c_void_p(core.data_ptr()), fptr,
                                        ctypes.c_void_p(dxhat.data_ptr()),
                                        ctypes.c_void_p(dcore.data_ptr() if dcore is not None else None), dptr,
                                        ctypes.c_void_p(ws.data_ptr()), need, ctypes.c_void_p(_stream(stream))))
    return dcore, dfs


class TuckerReconstruct(torch.autograd.Function):
    """X~ = (U_0, ..., U_{d-1}) . G with the hand-written adjoint.

    Saves only G and the U_n; the backward recomputes every partial product."""

    @staticmethod
    def forward(ctx, core, *factors):
        core = core.contiguous()
        factors = [f.contiguous() for f in factors]
        ctx.save_for_backward(core, *factors)
        return reconstruct(core, factors)

    @staticmethod
    def backward(ctx, grad_out):
        core, *factors = ctx.saved_tensors
        need_core = ctx.needs_input_grad[0]
        need_f = list(ctx.needs_input_grad[1:])
        dcore, dfs = reconstruct_backward(core, factors, grad_out.contiguous(), need_core, need_f)
        return (dcore, *dfs)


def tucker_reconstruct(core, *factors):
    return TuckerReconstruct.apply(core, *factors)


from .batched import BatchPlan, sthosvd_batched  # noqa: E402  (after the ctypes definitions)


# ------------------------------------------------------------- core quantization
@dataclass
class QuantStream:
    words: torch.Tensor          # int32 device tensor holding the 32-bit stream words
    k: Optional[int]             # scale exponent (None for an all-zero core)
    plane: int                   # breakpoint plane P (64: nothing encoded)
    count: int                   # coefficients encoded on plane P
    n: int
    block_len: int
    nblocks: int
    sse: float                   # |B - B~|^2 at the breakpoint (core units)
    status: int


def _quantize_launch(core: torch.Tensor, target_sse: float, block_len: int, stream=None):
    """Queues atc_quantize_core; returns (stream buffer of the maximal size, device info record)."""
    lib = load()
    _require_gpu(core, "core")
    n = core.numel()
    cap = lib.atc_quantize_max_words(n, int(block_len))
    wsz = lib.atc_quantize_workspace_size(n, int(block_len))
    if cap == 0 or wsz == 0:
        _check(-1)
    enc = torch.empty(cap, dtype=torch.int32, device=core.device)
    ws = torch.empty(wsz, dtype=torch.uint8, device=core.device)
    info_d = torch.empty(ctypes.sizeof(QuantInfo), dtype=torch.uint8, device=core.device)
    dt = ATC_F64 if core.dtype == torch.float64 else ATC_F32
    _check(lib.atc_quantize_core(ctypes.c_void_p(core.data_ptr()), dt, n, float(target_sse), int(block_len),
                                 ctypes.c_void_p(enc.data_ptr()), cap, ctypes.c_void_p(info_d.data_ptr()),
                                 ctypes.c_void_p(ws.data_ptr()), wsz, ctypes.c_void_p(_stream(stream))))
    return enc, info_d


def _quantize_finish(enc: torch.Tensor, info_d: torch.Tensor) -> QuantStream:
    """Reads the device record back (waits for the stream that wrote it)."""
    raw = bytes(info_d.cpu().numpy().tobytes())
    return _quantize_stream(enc, QuantInfo.from_buffer_copy(raw))


def _quantize_stream(enc: torch.Tensor, info: QuantInfo) -> QuantStream:
    """The stream of a quantization from its host copy of the record."""
    if info.status not in (0,):
        raise AtcError(info.status, "quantization of the core failed (device status)")
    return QuantStream(words=enc[: info.words], k=None if info.k == QUANT_KZERO else int(info.k), plane=int(info.plane),
                       count=int(info.count), n=int(info.n), block_len=int(info.block_len),
                       nblocks=int(info.nblocks), sse=float(info.sse), status=int(info.status))


def quantize_core(core: torch.Tensor, target_sse: float, block_len: int = 1024, stream=None) -> QuantStream:
    """Bit-plane quantization and encoding of `core` (vectorised in C order);
    see atc_quantize_core.  Reads the device record back (one synchronisation
    of `stream`)."""
    return _quantize_finish(*_quantize_launch(core, target_sse, block_len, stream))


def _dequantize_launch(words: torch.Tensor, n: int, block_len: int, dtype, status: torch.Tensor,
                       stream=None) -> torch.Tensor:
    """Queues atc_dequantize_core; the decoder's flags are OR-ed into `status`
    (a device int32), read by the caller."""
    lib = load()
    if not isinstance(words, torch.Tensor) or not words.is_cuda or words.dtype != torch.int32:
        raise ValueError("words must be an int32 GPU tensor")
    wsz = lib.atc_dequantize_workspace_size(int(n), int(block_len))
    if wsz == 0:
        _check(-1)
    ws = torch.empty(wsz, dtype=torch.uint8, device=words.device)
    out = torch.empty(int(n), dtype=dtype, device=words.device)
    dt = ATC_F64 if dtype == torch.float64 else ATC_F32
    _check(lib.atc_dequantize_core(ctypes.c_void_p(words.data_ptr()), int(n), int(block_len), dt,
                                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(status.data_ptr()),
                                   ctypes.c_void_p(ws.data_ptr()), wsz, ctypes.c_void_p(_stream(stream))))
    return out


def dequantize_core(words: torch.Tensor, n: int, block_len: int, dtype=torch.float32, stream=None) -> torch.Tensor:
    """Decoded core (n values, vectorised) of a stream; see atc_dequantize_core."""
    status = torch.zeros(1, dtype=torch.int32, device=words.device)
    out = _dequantize_launch(words, n, block_len, dtype, status, stream)
    if int(status.item()) != 0:
        raise AtcError(-7, "damaged stream: block fields do not match their planes")
    return out


# ------------------------------------------- factor representation, error model
def _ptr_or_null(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


def factor_householder(U: torch.Tensor, sigma2: Optional[torch.Tensor] = None, stream=None):
    """(coef float64, signs int32, U' = U diag(signs)) of a factor with
    orthonormal columns; see atc_factor_householder."""
    lib = load()
    _require_gpu(U, "U")
    n, r = int(U.shape[0]), int(U.shape[1])
    wsz = lib.atc_householder_workspace_size(n, r)
    if wsz == 0:
        _check(-1)
    if sigma2 is not None and (sigma2.dtype != torch.float64 or sigma2.numel() != r or not sigma2.is_cuda):
        raise ValueError("sigma2 must be a float64 GPU tensor of r entries")
    ws = torch.empty(wsz, dtype=torch.uint8, device=U.device)
    ncoef = n * r - r * (r + 1) // 2
    coef = torch.empty(max(1, ncoef), dtype=torch.float64, device=U.device)
    signs = torch.empty(r, dtype=torch.int32, device=U.device)
    up = torch.empty_like(U)
    dt = ATC_F64 if U.dtype == torch.float64 else ATC_F32
    _check(lib.atc_factor_householder(ctypes.c_void_p(U.data_ptr()), dt, n, r,
                                      _ptr_or_null(sigma2.contiguous() if sigma2 is not None else None),
                                      _ptr_or_null(coef), _ptr_or_null(signs), _ptr_or_null(up),
                                      ctypes.c_void_p(ws.data_ptr()), wsz, ctypes.c_void_p(_stream(stream))))
    return coef[:ncoef], signs, up


def factor_weight_coefficients(coef: torch.Tensor, sigma2: torch.Tensor, n: int, r: int, stream=None) -> torch.Tensor:
    """Scales unweighted reflector entries in place by sqrt(2 alpha_j); see
    atc_factor_weight_coefficients."""
    lib = load()
    if coef.dtype != torch.float64 or not coef.is_cuda or not coef.is_contiguous():
        raise ValueError("coef must be a contiguous float64 GPU tensor")
    if sigma2.dtype != torch.float64 or sigma2.numel() != int(r) or not sigma2.is_cuda:
        raise ValueError("sigma2 must be a float64 GPU tensor of r entries")
    if coef.numel() != int(n) * int(r) - int(r) * (int(r) + 1) // 2:
        raise ValueError("coef must hold n r - r (r + 1) / 2 entries")
    if coef.numel() == 0:
        return coef
    _check(lib.atc_factor_weight_coefficients(ctypes.c_void_p(coef.data_ptr()),
                                              ctypes.c_void_p(sigma2.contiguous().data_ptr()), int(n), int(r),
                                              ctypes.c_void_p(_stream(stream))))
    return coef


def factor_from_householder(coef: torch.Tensor, sigma2: Optional[torch.Tensor], n: int, r: int,
                            dtype=torch.float32, stream=None) -> torch.Tensor:
    """U' (n x r) from stored reflector entries; see atc_factor_from_householder."""
    lib = load()
    if coef.dtype != torch.float64 or not coef.is_cuda:
        raise ValueError("coef must be a float64 GPU tensor")
    wsz = lib.atc_householder_workspace_size(int(n), int(r))
    if wsz == 0:
        _check(-1)
    ws = torch.empty(wsz, dtype=torch.uint8, device=coef.device)
    out = torch.empty((int(n), int(r)), dtype=dtype, device=coef.device)
    if coef.numel() == 0:  # nothing stored (r = n = 1): any non-NULL pointer
        coef = torch.zeros(1, dtype=torch.float64, device=out.device)
    dt = ATC_F64 if dtype == torch.float64 else ATC_F32
    _check(lib.atc_factor_from_householder(ctypes.c_void_p(coef.data_ptr()),
                                           _ptr_or_null(sigma2.contiguous() if sigma2 is not None else None),
                                           int(n), int(r), dt, ctypes.c_void_p(out.data_ptr()),
                                           ctypes.c_void_p(ws.data_ptr()), wsz, ctypes.c_void_p(_stream(stream))))
    return out


def core_slice_norms(core: torch.Tensor, stream=None) -> List[torch.Tensor]:
    """Squared slice norms of the core per mode (float64 GPU tensors); see atc_core_slice_norms."""
    lib = load()
    _require_gpu(core, "core")
    s = _shape(list(core.shape), core.dtype)
    cnt = lib.atc_core_slice_norms_count(ctypes.byref(s))
    out = torch.empty(cnt, dtype=torch.float64, device=core.device)
    _check(lib.atc_core_slice_norms(ctypes.c_void_p(core.data_ptr()), ctypes.byref(s),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream(stream))))
    return list(torch.split(out, [int(n) for n in core.shape]))


def core_apply_signs(core: torch.Tensor, signs: Sequence[torch.Tensor], stream=None) -> torch.Tensor:
    """Flips the core's slices in place by the per-mode signs; see atc_core_apply_signs."""
    lib = load()
    _require_gpu(core, "core")
    s = _shape(list(core.shape), core.dtype)
    allsg = torch.cat([g.to(torch.int32) for g in signs]).contiguous()
    if allsg.numel() != sum(int(n) for n in core.shape):
        raise ValueError("one sign per slice of every mode")
    _check(lib.atc_core_apply_signs(ctypes.c_void_p(core.data_ptr()), ctypes.byref(s),
                                    ctypes.c_void_p(allsg.data_ptr()), ctypes.c_void_p(_stream(stream))))
    return core


def _factor_error_launch(U: torch.Tensor, Uq: torch.Tensor, sigma2: torch.Tensor, out: torch.Tensor, stream=None):
    """Queues atc_factor_error_term into out (one float64 on the device)."""
    lib = load()
    _require_gpu(U, "U")
    _require_gpu(Uq, "Uq")
    if U.shape != Uq.shape or U.dtype != Uq.dtype:
        raise ValueError("U and Uq must match")
    dt = ATC_F64 if U.dtype == torch.float64 else ATC_F32
    _check(lib.atc_factor_error_term(ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(Uq.data_ptr()), dt,
                                     int(U.shape[0]), int(U.shape[1]), ctypes.c_void_p(sigma2.contiguous().data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream(stream))))


def factor_error_term(U: torch.Tensor, Uq: torch.Tensor, sigma2: torch.Tensor, stream=None) -> float:
    """|dU Sigma|_F^2 of one factor (reads the device result back); see atc_factor_error_term."""
    out = torch.empty(1, dtype=torch.float64, device=U.device)
    _factor_error_launch(U, Uq, sigma2, out, stream)
    return float(out.item())


# ------------------------------------------------------------- hybrid compressor
@dataclass
class Compressed:
    tucker: Tucker                     # the ST-HOSVD (core and factors before quantization)
    core_stream: QuantStream           # the quantized core (slices flipped by the factor signs)
    factor_coef: List[torch.Tensor]    # weighted reflector entries per mode (before quantization)
    factor_streams: List[Optional[QuantStream]]  # their quantized streams (None: nothing to store)
    signs: List[torch.Tensor]
    sigma2: List[torch.Tensor]         # squared slice norms of the quantized core, per mode
    core_q: torch.Tensor               # dequantized core
    factors_q: List[torch.Tensor]      # factors rebuilt from the quantized reflectors
    factors_signed: List[torch.Tensor] # U diag(signs): the factors the quantized ones approximate
    predicted_sse: float               # eq. (total_error_approximation)
    terms: dict
    target_sse: float


def compress(x: torch.Tensor, rel_error: float = 1e-3, rtmss: float = 0.5, precision: str = "bf16x3",
             block_len: int = 1024, factor_share: float = 0.01, stream=None) -> Compressed:
    """The hybrid truncation of Section 4.1.3 end to end on the GPU: ST-HOSVD to
    rtmss * (rel_error |x|)^2, then one atc_hybrid_quantize call: the core
    quantized (Sections 3.3, 4.2, 4.3) to the rest of the target, each factor
    in its Householder form with the weights of supplement S.2 quantized to
    factor_share of the target split over the modes, and the terms of eq.
    (total_error_approximation).  This function allocates the outputs, forms
    the targets and reads the device records back once, at the end."""
    lib = load()
    t = sthosvd(x, rel_error, precision, rtmss=rtmss, stream=stream)
    d = len(t.ranks)
    target = rel_error * rel_error * t.norm2
    core = t.core.contiguous()
    facs = [f.contiguous() for f in t.factors]
    dev = x.device
    ranks = [int(r) for r in t.ranks]
    ns = [int(f.shape[0]) for f in facs]
    cs = _shape(ranks, core.dtype)
    n_arr = (ctypes.c_int64 * d)(*ns)
    wsz = lib.atc_hybrid_workspace_size(ctypes.byref(cs), n_arr, int(block_len))
    if wsz == 0:
        _check(-1)
    total = core.numel()
    out = HybridOut()
    keep = []  # every tensor the call writes, alive until the readback

    def buf(count, dtype):
        tt = torch.empty(max(1, int(count)), dtype=dtype, device=dev)
        keep.append(tt)
        return tt

    # the device records in one buffer, read back with one copy: d + 1 stream
    # records, d error terms, the decoders' status
    qsz = ctypes.sizeof(QuantInfo)
    rec = buf((d + 1) * qsz + 8 * d + 8, torch.uint8)
    core_info = rec[0:qsz]
    fterm = rec[(d + 1) * qsz:(d + 1) * qsz + 8 * d].view(torch.float64)
    status = rec[(d + 1) * qsz + 8 * d:(d + 1) * qsz + 8 * d + 4].view(torch.int32)
    core_enc = buf(lib.atc_quantize_max_words(total, int(block_len)), torch.int32)
    core_q = buf(total, core.dtype)
    sigma2 = buf(sum(ranks), torch.float64)
    signs_all = buf(sum(ranks), torch.int32)
    out.core_enc, out.core_info, out.core_q = core_enc.data_ptr(), core_info.data_ptr(), core_q.data_ptr()
    out.sigma2, out.signs = sigma2.data_ptr(), signs_all.data_ptr()
    out.factor_term, out.status = fterm.data_ptr(), status.data_ptr()
    signed, coefs, fencs, finfos, facs_q, ncoef = [], [], [], [], [], []
    for k in range(d):
        n, r = ns[k], ranks[k]
        e = n * r - r * (r + 1) // 2
        ncoef.append(e)
        signed.append(buf(n * r, core.dtype).view(n, r))
        coefs.append(buf(e, torch.float64))
        facs_q.append(buf(n * r, core.dtype).view(n, r))
        if e > 0:
            fencs.append(buf(lib.atc_quantize_max_words(e, int(block_len)), torch.int32))
            finfos.append(rec[(k + 1) * qsz:(k + 2) * qsz])
            out.factor_enc[k], out.factor_info[k] = fencs[-1].data_ptr(), finfos[-1].data_ptr()
        else:
            fencs.append(None)
            finfos.append(None)
        out.factor_signed[k], out.factor_coef[k] = signed[k].data_ptr(), coefs[k].data_ptr()
        out.factor_q[k] = facs_q[k].data_ptr()
    ws = buf(wsz, torch.uint8)
    fptrs = (ctypes.c_void_p * d)(*[f.data_ptr() for f in facs])
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib.atc_hybrid_quantize(ctypes.c_void_p(core.data_ptr()), ctypes.byref(cs), fptrs, n_arr,
                                   float(target - t.sse_pred), float(factor_share * target / d), int(block_len),
                                   ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()), wsz,
                                   ctypes.c_void_p(_stream(st))))
    raw = rec.cpu().numpy().tobytes()  # waits for the stream
    infos = [QuantInfo.from_buffer_copy(raw[i * qsz:(i + 1) * qsz]) for i in range(d + 1)]
    cs_q = _quantize_stream(core_enc, infos[0])
    fstreams = [_quantize_stream(fencs[k], infos[k + 1]) if ncoef[k] > 0 else None for k in range(d)]
    if int(np.frombuffer(raw, dtype=np.int32, count=1, offset=(d + 1) * qsz + 8 * d)[0]) != 0:
        raise AtcError(-7, "damaged stream: block fields do not match their planes")
    fterms = [float(v) for v in np.frombuffer(raw, dtype=np.float64, count=d, offset=(d + 1) * qsz)]
    signs = list(torch.split(signs_all, ranks))
    s2 = list(torch.split(sigma2, ranks))
    pred = t.sse_pred + cs_q.sse + sum(fterms)
    return Compressed(tucker=t, core_stream=cs_q, factor_coef=[coefs[k][:ncoef[k]] for k in range(d)],
                      factor_streams=fstreams, signs=signs, sigma2=s2, core_q=core_q.view(*ranks),
                      factors_q=facs_q, factors_signed=signed, predicted_sse=pred,
                      terms={"sthosvd": t.sse_pred, "core": cs_q.sse, "factors": fterms}, target_sse=target)


def decompress(c: Compressed, stream=None) -> torch.Tensor:
    """A~ = (U~_0, ..., U~_{d-1}) . B~ from the quantized core and factors."""
    return reconstruct(c.core_q.contiguous(), [f.contiguous() for f in c.factors_q], stream=stream)
