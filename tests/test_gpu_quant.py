"""GPU parity of the core quantization and encoding (atc_quantize_core /
atc_dequantize_core, through the C ABI) with the oracle of Section 3.3
(TTHRESH bit planes), Section 4.2 (blocks, per-block breakpoints) and Section
4.3 (dequantization correction in the error tracking).

Bars: integer and bit work is bit-exact -- the scale exponent, the breakpoint
(plane, position), every word of the stream, and the decoded values (both
sides scale the same integers by 2^-k and round once); the reported error
agrees with the oracle's exact one to 1e-12 relative (one rounding of a
192-bit integer on the device).  Cores: synthetic hot-corner tensors
(entries decaying away from the origin, as an ST-HOSVD core) with ragged last
blocks, several block lengths and targets from 'nothing encoded' to 'every
bit', the all-zero core, and the core of the 512^3 field's ST-HOSVD at
RTMSS = 0.5 with the hybrid target of Section 4.1.3 (total SSE target minus
the ST-HOSVD's).
"""
import numpy as np
import pytest
import torch

import paper_2107_01384_amd as atc
import synth
from gpu_helpers import log
from oracle import quant

pytestmark = pytest.mark.gpu


def _hot_corner(shape, seed, tau=4.0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    return x * np.exp(-sum(grids) / tau)


def _check(values, dtype, block_len, target):
    """GPU stream and decoding against the oracle, bit for bit."""
    core = torch.from_numpy(np.ascontiguousarray(values)).to("cuda", dtype)
    v64 = core.double().cpu().numpy()          # the values the GPU sees, exactly
    st = atc.quantize_core(core, target, block_len)
    words_g = st.words.cpu().numpy().view(np.uint32)
    words_o = quant.encode(v64, target, block_len)
    h = quant.decode(words_o)[0]
    log("quant %s %s L=%d target %.3e: k %s plane %d count %d words %d (oracle k %s plane %d count %d words %d)"
        % (values.shape, dtype, block_len, target, st.k, st.plane, st.count, words_g.size, h["k"], h["P"],
           h["count"], words_o.size))
    assert (st.k, st.plane, st.count, st.n, st.nblocks) == (h["k"], h["P"], h["count"], h["n"], h["nblocks"])
    assert words_g.size == words_o.size
    assert np.array_equal(words_g, words_o)
    sse_o = quant.core_sse(v64, words_o)
    assert abs(st.sse - sse_o) <= 1e-12 * max(sse_o, 1e-300), (st.sse, sse_o)
    # decoding: the GPU's of its own stream, against the oracle's values
    for odt in (torch.float64, torch.float32):
        out = atc.dequantize_core(st.words, st.n, block_len, odt).cpu().numpy()
        ref = quant.dequantize(words_o)
        ref = ref if odt == torch.float64 else ref.astype(np.float32)
        assert np.array_equal(out, ref), odt
    return st, v64, words_o


CASES = [
    ((5, 4, 3), torch.float64, 7, 1e-6),
    ((5, 4, 3), torch.float32, 1, 1e-3),
    ((33, 31, 29), torch.float64, 64, 1e-7),
    ((20, 17, 20), torch.float32, 1024, 1e-5),
    ((40, 40, 40), torch.float32, 4096, 1e-6),
    ((7, 9, 11, 13), torch.float64, 100, 1e-8),
    ((257,), torch.float32, 3, 1e-4),
    ((2, 3), torch.float64, 4096, 1e-12),
]


@pytest.mark.parametrize("shape,dtype,block_len,rel", CASES)
def test_quant_parity(shape, dtype, block_len, rel):
    v = _hot_corner(shape, sum(shape) + block_len)
    target = rel * float(np.sum(v * v))
    _check(v, dtype, block_len, target)


def test_quant_degenerate_targets_and_cores():
    v = _hot_corner((9, 8, 7), 5)
    # target at or above the error of encoding nothing: nothing encoded
    st, _, _ = _check(v, torch.float64, 50, 2.0 * float(np.sum(v * v)))
    assert st.plane == 64 and st.count == 0
    # below zero: every bit; decoding gives the core up to the rounding to integers
    st, v64, _ = _check(v, torch.float64, 50, -1.0)
    assert st.plane == 0 and st.count == v.size
    out = atc.dequantize_core(st.words, st.n, 50, torch.float64).cpu().numpy()
    assert np.max(np.abs(out - v64.ravel())) <= 2.0 ** (-st.k - 1)
    # zero target: every error-carrying bit (plane 0 reaches zero error)
    _check(v, torch.float32, 64, 0.0)
    # all-zero core
    st, _, _ = _check(np.zeros((4, 5)), torch.float32, 8, 1e-3)
    assert st.k is None and st.plane == 64
    # a single coefficient
    _check(np.array([-3.25]), torch.float64, 1, 1e-9)


def test_quant_nonfinite_core_reports():
    v = _hot_corner((6, 6), 2)
    v[2, 3] = np.inf
    core = torch.from_numpy(v).cuda()
    with pytest.raises(atc.AtcError) as e:
        atc.quantize_core(core, 1e-3, 16)
    assert e.value.status == -6


def test_quant_sthosvd_core_field512_hybrid():
    """The 512^3 field's ST-HOSVD at eps = 1e-3 with RTMSS = 0.5 (Section 4.1.3):
    the core quantized to the rest of the total SSE target.  With orthonormal
    factors the truncation error lies outside the factors' span and the
    quantization error inside it, so |A - A~|^2 = |A - A^|^2 + |B - B~|^2: the
    measured growth of the error must equal the reported quantization error."""
    eps = 1e-3
    x = torch.from_numpy(synth.field((512,) * 3, 0)).cuda()
    t = atc.sthosvd(x, eps, "bf16x3", rtmss=0.5)
    torch.cuda.synchronize()
    budget = eps * eps * t.norm2
    target = budget - t.sse_pred
    log("512^3 rtmss 0.5: ranks %s, ST-HOSVD SSE %.4e of budget, core target %.4e" % (
        t.ranks, t.sse_pred / budget, target))
    st, v64, words_o = _check(t.core.contiguous().cpu().numpy(), torch.float32, 1024, target)
    assert st.sse <= target
    facs = [f.contiguous() for f in t.factors]

    def sq_err(core):
        xh = atc.reconstruct(core, facs)
        return float(((x.double() - xh.double()) ** 2).sum())

    e_trunc = sq_err(t.core.contiguous())
    deq = atc.dequantize_core(st.words, st.n, 1024, torch.float32).view(*t.ranks)
    e_tot = sq_err(deq)
    log("  |A - A^|^2 / budget %.6f (predicted %.6f), |A - A~|^2 / budget %.6f, growth / quantization SSE %.6f"
        % (e_trunc / budget, t.sse_pred / budget, e_tot / budget, (e_tot - e_trunc) / st.sse))
    assert abs((e_tot - e_trunc) - st.sse) <= 1e-3 * st.sse
    assert e_tot <= 1.02 ** 2 * budget
