"""atc_reconstruct_noalloc (intermediates in the library's static device
scratch, nothing allocated by the call) against atc_reconstruct (caller
workspace), through the C ABI: element by element on two calls in a row, the
second on a smaller problem, in float32 and float64; sizes beyond the
scratch are refused on the host before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2107_01384_amd as atc
from gpu_helpers import log

pytestmark = pytest.mark.gpu


def _model(dims, ranks, dtype, seed):
    rng = np.random.default_rng(seed)
    core = torch.from_numpy(rng.standard_normal(ranks)).to("cuda", dtype)
    facs = [torch.from_numpy(np.linalg.qr(rng.standard_normal((n, r)))[0]).to("cuda", dtype)
            for n, r in zip(dims, ranks)]
    return core, facs


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_workspace_call_twice(dtype):
    cases = [((96, 80, 72, 6), (20, 17, 12, 3)), ((33, 17, 40), (5, 9, 7))]
    for i, (dims, ranks) in enumerate(cases):
        log("noalloc reconstruct", dims, ranks, dtype)
        core, facs = _model(dims, ranks, dtype, 40 + i)
        ref = atc.reconstruct(core, facs)
        out = torch.full(dims, float("nan"), dtype=dtype, device="cuda")
        atc.reconstruct_noalloc(core, facs, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (dims, float((out - ref).abs().max()))


def test_noalloc_refuses_beyond_scratch():
    lib = atc.load()
    dims, ranks = (512, 512, 512), (64, 64, 64)
    s = atc._shape(dims, torch.float32)
    ra = atc._ranks_arr(ranks)
    need = lib.atc_reconstruct_workspace_size(ctypes.byref(s), ra)
    assert need > (64 << 20)
    fptr = (ctypes.c_void_p * 3)(1, 1, 1)
    st = lib.atc_reconstruct_noalloc(ctypes.byref(s), ra, ctypes.c_void_p(1), fptr, ctypes.c_void_p(1),
                                     ctypes.c_void_p(None))
    assert st == -2 and b"scratch" in lib.atc_last_error()
