"""Pins for the oracle's reconstruction, decompression order and gradient.

* Section 4.1.1 decompression cost and exhaustive order search: hand-derived values.
* Reconstruction = expanding every mode by its factor: checked against einsum.
* Gradient of L = 0.5 |X~ - Y|^2: X~ is linear in each block (G or one U_n), so L
  is exactly quadratic along a direction that moves one block, and the central
  difference (L(t + h V) - L(t - h V)) / 2h equals <dL, V> up to rounding for any h.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import load_golden


def test_decompression_order_costs():
    g = load_golden("recon_order.json")
    order, cost = oracle.reconstruct_order(g["dims"], g["ranks"])
    assert order == g["best_order"] and cost == g["best_cost"]
    assert oracle.reconstruct_cost(g["dims"], g["ranks"], g["worst_order"]) == g["worst_cost"]
    import itertools
    worst = max(oracle.reconstruct_cost(g["dims"], g["ranks"], p) for p in itertools.permutations(range(4)))
    assert worst == g["worst_cost"]


def test_reconstruct_matches_einsum():
    rng = np.random.default_rng(21)
    core = rng.standard_normal((2, 3, 4, 2))
    facs = [rng.standard_normal((n, r)) for n, r in zip((5, 6, 7, 3), core.shape)]
    ref = np.einsum("abcd,ia,jb,kc,ld->ijkl", core, *facs)
    for order in (None, [3, 2, 1, 0], [1, 3, 0, 2]):
        assert np.allclose(oracle.reconstruct(core, facs, order), ref, rtol=1e-13, atol=1e-13)


def _problem(seed=22):
    dims, ranks = (6, 5, 4, 3), (3, 2, 3, 2)
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(ranks)
    facs = [np.linalg.qr(rng.standard_normal((n, r)))[0] for n, r in zip(dims, ranks)]
    y = rng.standard_normal(dims)
    return core, facs, y


def test_gradient_is_exact_central_difference():
    core, facs, y = _problem()
    loss, dg, dus = oracle.loss_and_grad(core, facs, y)
    rng = np.random.default_rng(23)
    h = 1e-3

    def L(c, f):
        return 0.5 * oracle.norm2(oracle.reconstruct(c, f) - y)

    assert abs(L(core, facs) - loss) <= 1e-14 * loss
    for _ in range(4):
        v = rng.standard_normal(core.shape)
        fd = (L(core + h * v, facs) - L(core - h * v, facs)) / (2 * h)
        assert abs(fd - np.sum(dg * v)) <= 1e-9 * max(1.0, abs(fd))
        for n in range(4):
            vn = rng.standard_normal(facs[n].shape)
            fp = [f.copy() for f in facs]
            fm = [f.copy() for f in facs]
            fp[n] += h * vn
            fm[n] -= h * vn
            fd = (L(core, fp) - L(core, fm)) / (2 * h)
            assert abs(fd - np.sum(dus[n] * vn)) <= 1e-9 * max(1.0, abs(fd))


def test_gradient_matches_explicit_unfolding_formula():
    """dL/dU_n = D_(n) W_(n)^T with W the core expanded in every mode but n;
    dL/dG = D expanded back by the transposed factors (einsum route)."""
    core, facs, y = _problem(24)
    loss, dg, dus = oracle.loss_and_grad(core, facs, y)
    xh = np.einsum("abcd,ia,jb,kc,ld->ijkl", core, *facs)
    d = xh - y
    assert np.allclose(dg, np.einsum("ijkl,ia,jb,kc,ld->abcd", d, *facs), rtol=1e-12, atol=1e-12)
    w0 = np.einsum("abcd,jb,kc,ld->ajkl", core, facs[1], facs[2], facs[3])
    assert np.allclose(dus[0], np.einsum("ijkl,ajkl->ia", d, w0), rtol=1e-12, atol=1e-12)
    w3 = np.einsum("abcd,ia,jb,kc->ijkd", core, facs[0], facs[1], facs[2])
    assert np.allclose(dus[3], np.einsum("ijkl,ijkd->ld", d, w3), rtol=1e-12, atol=1e-12)


def test_sthosvd_then_reconstruct_error_matches_prediction():
    x = synth.field((16, 24, 20), 9).astype(np.float64)
    for eps in (1e-2, 1e-3):
        t = oracle.sthosvd(x, eps)
        err = oracle.rel_error(x, t.core, t.factors)
        assert abs(err - np.sqrt(t.sse_pred / t.norm2)) <= 1e-8 * eps
