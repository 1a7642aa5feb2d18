"""GPU parity of the Householder factor representation (supplement S.2) and of
the error-model terms (Section 4.1.3, eq. total_error_approximation), through
the C ABI, against oracle/householder.py.

Bars: FP64 on both sides with different summation orders, so the weighted
coefficients and the rebuilt factors agree to 1e-12 (relative to their
largest entry), the column signs exactly; the slice norms and the factor error
term to 1e-12 relative.  Factors: random orthonormal n x r (r = 1, r = n,
ragged sizes) and the 512^3 field's ST-HOSVD factors with the slice norms of
its core; float32 and float64.
"""
import numpy as np
import pytest
import torch

import paper_2107_01384_amd as atc
import synth
from gpu_helpers import log
from oracle import householder as hh

pytestmark = pytest.mark.gpu


def _orth(n, r, seed):
    rng = np.random.default_rng(seed)
    return np.linalg.qr(rng.standard_normal((n, r)))[0]


CASES = [(1, 1), (6, 6), (64, 8), (200, 20), (512, 18), (300, 64), (1000, 3)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,r", CASES)
def test_householder_parity(n, r, dtype):
    U = _orth(n, r, n * 7 + r)
    rng = np.random.default_rng(n + r)
    s2 = np.sort(rng.uniform(0.01, 100.0, r))[::-1].copy()
    Ud = torch.from_numpy(U).to("cuda", dtype)
    U64 = Ud.double().cpu().numpy()          # the values the GPU sees
    for weights in (None, s2):
        log("householder n %d r %d %s weights %s" % (n, r, dtype, weights is not None))
        sd = None if weights is None else torch.from_numpy(weights).cuda()
        coef, signs, Up = atc.factor_householder(Ud, sd)
        c_o, s_o, Up_o = hh.encode(U64, weights)
        assert np.array_equal(signs.cpu().numpy(), s_o.astype(np.int32))
        cg = coef.cpu().numpy()
        assert cg.size == hh.ncoef(n, r)
        scale = max(1.0, np.abs(c_o).max(initial=0.0))
        assert np.abs(cg - c_o).max(initial=0.0) <= 1e-12 * scale
        assert np.array_equal(Up.double().cpu().numpy(), (U64 * s_o).astype(np.float64) if dtype == torch.float64
                              else (U64 * s_o).astype(np.float32).astype(np.float64))
        # decoding: the GPU's from its own coefficients and the oracle's from the same numbers
        Ur = atc.factor_from_householder(coef, sd, n, r, torch.float64).cpu().numpy()
        Ur_o = hh.decode(cg, n, r, weights)
        assert np.abs(Ur - Ur_o).max() <= 1e-12
        # the reflectors rebuild an orthonormal matrix: the input itself up to
        # its own orthonormality defect (float32 input carries ~1e-8)
        defect = np.abs(U64.T @ U64 - np.eye(r)).max()
        assert np.abs(Ur - U64 * s_o).max() <= 1e-12 * max(1, r) + 4.0 * defect


@pytest.mark.parametrize("n,r", [(1, 1), (6, 6), (200, 20), (512, 18), (1000, 3)])
def test_weighting_stored_entries(n, r):
    """Unweighted entries scaled in place (atc_factor_weight_coefficients)
    against the oracle's weighted encoding, and the entries of U diag(s) for
    random signs s against those of U (supplement S.2: the same reflectors)."""
    U = _orth(n, r, 5 * n + r)
    rng = np.random.default_rng(3 * n + r)
    s2 = np.sort(rng.uniform(0.01, 100.0, r))[::-1].copy()
    Ud = torch.from_numpy(U).cuda()
    sd = torch.from_numpy(s2).cuda()
    log("weighting n %d r %d" % (n, r))
    coef, signs, _ = atc.factor_householder(Ud, None)
    flip = torch.from_numpy(np.where(rng.random(r) < 0.5, -1.0, 1.0)).cuda()
    coef_f, _, _ = atc.factor_householder((Ud * flip).contiguous(), None)
    assert torch.equal(coef, coef_f)
    atc.factor_weight_coefficients(coef, sd, n, r)
    c_o, _, _ = hh.encode(U, s2)
    cg = coef.cpu().numpy()
    scale = max(1.0, np.abs(c_o).max(initial=0.0))
    assert cg.size == c_o.size
    assert np.abs(cg - c_o).max(initial=0.0) <= 1e-12 * scale


def test_slice_norms_signs_and_factor_term_field512():
    """The 512^3 field's ST-HOSVD (eps 1e-3, RTMSS 0.5): slice norms of its core
    per mode, the core's slices flipped by the Householder signs of every
    factor (the reconstruction is unchanged), and |dU Sigma|^2 of a perturbed
    factor."""
    x = torch.from_numpy(synth.field((512,) * 3, 0)).cuda()
    t = atc.sthosvd(x, 1e-3, "bf16x3", rtmss=0.5)
    torch.cuda.synchronize()
    core = t.core.contiguous()
    s2 = atc.core_slice_norms(core)
    s2_o = hh.slice_norms2(core.double().cpu().numpy())
    for k in range(3):
        g = s2[k].cpu().numpy()
        assert np.abs(g - s2_o[k]).max() <= 1e-12 * s2_o[k].max()
    # Householder signs of every factor, applied to the factor and the core
    facs, signs = [], []
    for k, f in enumerate(t.factors):
        coef, sg, Up = atc.factor_householder(f.contiguous(), s2[k])
        facs.append(Up)
        signs.append(sg)
    flipped = core.clone()
    atc.core_apply_signs(flipped, signs)
    ref = core.double().cpu().numpy()
    for k in range(3):
        sh = [1, 1, 1]
        sh[k] = -1
        ref = ref * signs[k].cpu().numpy().astype(np.float64).reshape(sh)
    assert np.array_equal(flipped.double().cpu().numpy(), ref)
    a = atc.reconstruct(core, [f.contiguous() for f in t.factors])
    b = atc.reconstruct(flipped, facs)
    assert torch.equal(a, b) or float((a - b).abs().max()) <= 1e-6 * float(a.abs().max())
    # factor error term of a perturbed factor
    rng = np.random.default_rng(9)
    U0 = facs[0]
    Uq = U0 + torch.from_numpy(1e-4 * rng.standard_normal(tuple(U0.shape))).to("cuda", U0.dtype)
    term = atc.factor_error_term(U0, Uq, s2[0])
    term_o = hh.factor_error_term(U0.double().cpu().numpy(), Uq.double().cpu().numpy(), s2[0].cpu().numpy())
    assert abs(term - term_o) <= 1e-12 * term_o
