"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/atc.h declares, sizes its structs like the header, and rejects bad
arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest
import torch

import paper_2107_01384_amd as atc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "atc.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(atc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = atc.load()
    names = declared_symbols()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in atc.SIGNATURES}
    assert set(names) == bound


def test_struct_sizes_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "%s"\nint main(){printf("%%zu %%zu %%zu %%zu %%zu %%zu",'
                   'sizeof(atc_sthosvd_opts),sizeof(atc_result),sizeof(atc_block_result),sizeof(atc_shape),'
                   'sizeof(atc_quant_info),sizeof(atc_hybrid_out));}\n' % HEADER)
    exe = tmp_path / "sz"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert [int(v) for v in out] == [ctypes.sizeof(atc.Opts), ctypes.sizeof(atc.Result),
                                     ctypes.sizeof(atc.BlockResult), ctypes.sizeof(atc.Shape),
                                     ctypes.sizeof(atc.QuantInfo), ctypes.sizeof(atc.HybridOut)]


def _shape(dims, dtype=0):
    s = atc.Shape()
    s.ndim = len(dims)
    s.dtype = dtype
    for i, n in enumerate(dims):
        s.dims[i] = n
    return s


def test_argument_validation_without_device():
    lib = atc.load()
    o = atc.make_opts(1e-3)
    s = _shape([4, 5, 6])
    ws = lib.atc_sthosvd_workspace_size(ctypes.byref(s), ctypes.byref(o))
    assert ws > 0
    null = ctypes.c_void_p(None)
    facs = (ctypes.c_void_p * 3)(1, 1, 1)
    # NULL input
    st = lib.atc_sthosvd(null, ctypes.byref(s), ctypes.byref(o), ctypes.c_void_p(1), facs, None,
                         ctypes.c_void_p(1), ws, null)
    assert st == -1 and b"non-NULL" in lib.atc_last_error()
    # workspace too small
    st = lib.atc_sthosvd(ctypes.c_void_p(1), ctypes.byref(s), ctypes.byref(o), ctypes.c_void_p(1), facs, None,
                         ctypes.c_void_p(1), ws - 1, null)
    assert st == -3
    # bad shapes and options
    for bad in (_shape([4, 0, 6]), _shape([]), _shape([2] * 9 if False else [5, 5], dtype=7)):
        assert lib.atc_sthosvd(ctypes.c_void_p(1), ctypes.byref(bad), ctypes.byref(o), ctypes.c_void_p(1), facs,
                               None, ctypes.c_void_p(1), ws, null) == -1
    for kw in ({"rel_error": -1.0}, {"rtmss": 1.5}, {"order": [0, 0, 1]}, {"fixed_ranks": [5, 1, 1]},
               {"max_sweeps": -3}, {"eig_path": 3}, {"no_host_wait": True},
               {"no_host_wait": True, "fixed_ranks": [2, 2, 2], "profile": True}):
        args = {"rel_error": 1e-3}
        args.update(kw)
        ob = atc.make_opts(**args)
        assert lib.atc_sthosvd(ctypes.c_void_p(1), ctypes.byref(s), ctypes.byref(ob), ctypes.c_void_p(1), facs,
                               None, ctypes.c_void_p(1), ws, null) == -1, kw
    # bf16x3 needs float32 input; modes beyond 4096 are not built
    o3 = atc.make_opts(1e-3, "bf16x3")
    assert lib.atc_sthosvd(ctypes.c_void_p(1), ctypes.byref(_shape([4, 5], 1)), ctypes.byref(o3), ctypes.c_void_p(1),
                           facs, None, ctypes.c_void_p(1), ws, null) == -2
    assert lib.atc_sthosvd_workspace_size(ctypes.byref(_shape([5000, 2])), ctypes.byref(o)) == 0
    # atc_sthosvd_finish: only after a no-host-wait call, with the same workspace size
    res = atc.Result()
    assert lib.atc_sthosvd_finish(ctypes.byref(s), ctypes.byref(o), ctypes.c_void_p(1), ws, ctypes.byref(res),
                                  null) == -1
    # forced subspace path with a rank beyond its Ritz pairs: refused up front
    big = _shape([100, 90, 80])
    assert lib.atc_sthosvd_workspace_size(ctypes.byref(big), ctypes.byref(
        atc.make_opts(1e-3, fixed_ranks=[57, 5, 5], eig_path=2, no_host_wait=True))) == 0
    assert lib.atc_sthosvd_workspace_size(ctypes.byref(big), ctypes.byref(
        atc.make_opts(1e-3, fixed_ranks=[56, 5, 5], eig_path=2, no_host_wait=True))) > 0
    onw = atc.make_opts(1e-3, fixed_ranks=[2, 2, 2], no_host_wait=True)
    assert lib.atc_sthosvd_workspace_size(ctypes.byref(s), ctypes.byref(onw)) == ws
    assert lib.atc_sthosvd_finish(ctypes.byref(s), ctypes.byref(onw), ctypes.c_void_p(1), ws - 1,
                                  ctypes.byref(res), null) == -3
    # reconstruction: ranks outside [1, n]
    ra = (ctypes.c_int64 * 8)(3, 6, 2)
    assert lib.atc_reconstruct_workspace_size(ctypes.byref(s), ra) == 0
    ra = (ctypes.c_int64 * 8)(3, 5, 2)
    assert lib.atc_reconstruct_workspace_size(ctypes.byref(s), ra) > 0
    assert lib.atc_status_string(-5) == b"eigensolver did not converge"


def test_workspace_size_scales_with_tensor():
    lib = atc.load()
    o = atc.make_opts(1e-3, "bf16x3")
    small = lib.atc_sthosvd_workspace_size(ctypes.byref(_shape([64, 64, 64])), ctypes.byref(o))
    big = lib.atc_sthosvd_workspace_size(ctypes.byref(_shape([512, 512, 512])), ctypes.byref(o))
    assert big > 2 * 512 ** 3 * 4 > small


def test_quant_argument_validation_without_device():
    lib = atc.load()
    assert lib.atc_quantize_max_words(0, 64) == 0
    assert lib.atc_quantize_max_words(100, 5000) == 0
    cap = lib.atc_quantize_max_words(100, 64)
    wsz = lib.atc_quantize_workspace_size(100, 64)
    assert cap > 10 + 2 * 2 and wsz > 100 * 8
    one = ctypes.c_void_p(1)
    null = ctypes.c_void_p(None)
    assert lib.atc_quantize_core(one, 0, 0, 1.0, 64, one, cap, one, one, wsz, null) == -1
    assert lib.atc_quantize_core(one, 0, 100, 1.0, 5000, one, cap, one, one, wsz, null) == -2
    assert lib.atc_quantize_core(one, 0, 100, 1.0, 64, one, cap - 1, one, one, wsz, null) == -3
    assert lib.atc_quantize_core(one, 0, 100, 1.0, 64, one, cap, one, one, wsz - 1, null) == -3
    assert lib.atc_quantize_core(one, 0, 100, float("nan"), 64, one, cap, one, one, wsz, null) == -1
    assert lib.atc_quantize_core(null, 0, 100, 1.0, 64, one, cap, one, one, wsz, null) == -1
    assert lib.atc_quantize_core(one, 3, 100, 1.0, 64, one, cap, one, one, wsz, null) == -1
    dsz = lib.atc_dequantize_workspace_size(100, 64)
    assert dsz > 0
    assert lib.atc_dequantize_core(one, 100, 64, 0, one, null, one, dsz - 1, null) == -3
    assert lib.atc_dequantize_core(one, 100, 0, 0, one, null, one, dsz, null) == -2


def test_hybrid_argument_validation_without_device():
    """atc_hybrid_workspace_size / atc_hybrid_quantize reject bad shapes,
    block lengths and NULL buffers before touching a device."""
    lib = atc.load()
    cs = atc._shape([5, 4, 3], torch.float32)
    n = (ctypes.c_int64 * 3)(20, 16, 12)
    assert lib.atc_hybrid_workspace_size(ctypes.byref(cs), n, 64) > 0
    assert lib.atc_hybrid_workspace_size(ctypes.byref(cs), n, 0) == 0
    assert lib.atc_hybrid_workspace_size(ctypes.byref(cs), n, 5000) == 0
    bad = (ctypes.c_int64 * 3)(20, 3, 12)  # r_1 = 4 > n_1 = 3
    assert lib.atc_hybrid_workspace_size(ctypes.byref(cs), bad, 64) == 0
    big = atc._shape([300, 4, 3], torch.float32)  # r_0 > 256
    assert lib.atc_hybrid_workspace_size(ctypes.byref(big), (ctypes.c_int64 * 3)(400, 16, 12), 64) == 0
    out = atc.HybridOut()
    one = ctypes.c_void_p(1)
    facs = (ctypes.c_void_p * 3)(1, 1, 1)
    # NULL outputs are refused before any launch
    st = lib.atc_hybrid_quantize(one, ctypes.byref(cs), facs, n, 1.0, 1.0, 64, ctypes.byref(out), one, 1 << 30,
                                 ctypes.c_void_p(None))
    assert st == -1
