"""GPU parity of atc_reconstruct / atc_reconstruct_backward and the autograd
Function against the FP64 oracle (values and exact gradient)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2107_01384_amd as atc
from gpu_helpers import log, np64, to_dev

pytestmark = pytest.mark.gpu

CASES = [((6, 5, 4, 3), (3, 2, 3, 2)), ((70, 33, 9), (10, 33, 4)), ((130, 20), (7, 20)), ((17,), (5,)),
         ((40, 50, 3, 20), (8, 12, 3, 5)), ((20, 17, 64), (9, 7, 4)), ((10, 9, 96), (8, 8, 6)),
         ((12, 11, 40), (6, 5, 3)), ((30, 21, 17, 36), (5, 4, 3, 9)), ((30, 21, 17, 35), (5, 4, 3, 9))]


def _model(dims, ranks, seed):
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(ranks)
    facs = [np.linalg.qr(rng.standard_normal((n, r)))[0] for n, r in zip(dims, ranks)]
    return core, facs


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
@pytest.mark.parametrize("dims,ranks", CASES)
def test_reconstruct_parity(dims, ranks, dtype, tol):
    log("reconstruct", dims, ranks, dtype)
    core, facs = _model(dims, ranks, 5)
    ref = oracle.reconstruct(core, facs)
    out = atc.reconstruct(to_dev(core, dtype), [to_dev(f, dtype) for f in facs])
    torch.cuda.synchronize()
    got = np64(out)
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
@pytest.mark.parametrize("dims,ranks", CASES)
def test_backward_parity(dims, ranks, dtype, tol):
    log("backward", dims, ranks, dtype)
    core, facs = _model(dims, ranks, 6)
    y = np.random.default_rng(7).standard_normal(dims)
    loss, dg, dus = oracle.loss_and_grad(core, facs, y)
    xh = oracle.reconstruct(core, facs)
    dcore, dfs = atc.reconstruct_backward(to_dev(core, dtype), [to_dev(f, dtype) for f in facs],
                                          to_dev(xh - y, dtype))
    torch.cuda.synchronize()
    # norm-wise, and entry by entry against the largest entry of each output
    ratios = [np.abs(np64(dcore) - dg).max() / np.abs(dg).max()]
    assert np.linalg.norm(np64(dcore) - dg) <= tol * np.linalg.norm(dg)
    for n in range(len(dims)):
        assert np.linalg.norm(np64(dfs[n]) - dus[n]) <= tol * np.linalg.norm(dus[n])
        ratios.append(np.abs(np64(dfs[n]) - dus[n]).max() / np.abs(dus[n]).max())
    log("  entry-wise max error / max entry: dG %.2e, dU %s" % (ratios[0], ["%.2e" % r for r in ratios[1:]]))
    assert max(ratios) <= tol, ratios


def test_autograd_function_matches_oracle_and_saves_only_inputs():
    dims, ranks = (24, 20, 16, 12), (6, 5, 4, 3)
    core, facs = _model(dims, ranks, 8)
    y = np.random.default_rng(9).standard_normal(dims)
    loss_ref, dg, dus = oracle.loss_and_grad(core, facs, y)
    g = to_dev(core, torch.float64).requires_grad_(True)
    us = [to_dev(f, torch.float64).requires_grad_(True) for f in facs]
    yt = to_dev(y, torch.float64)
    xh = atc.tucker_reconstruct(g, *us)
    # only the inputs are saved for backward (no partial products)
    saved = xh.grad_fn.saved_tensors
    assert len(saved) == 1 + len(us)
    assert sum(t.numel() for t in saved) == g.numel() + sum(u.numel() for u in us)
    loss = 0.5 * ((xh - yt) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - loss_ref) <= 1e-12 * loss_ref
    assert np.allclose(np64(g.grad), dg, rtol=1e-11, atol=1e-11 * np.abs(dg).max())
    for n in range(4):
        assert np.allclose(np64(us[n].grad), dus[n], rtol=1e-11, atol=1e-11 * np.abs(dus[n]).max())


def test_autograd_directional_finite_differences_fp32():
    """FP32 GPU gradient against central differences of the FP64 loss (exact for a
    direction that moves one block, since the loss is quadratic along it)."""
    dims, ranks = (16, 12, 10, 8), (4, 3, 3, 2)
    core, facs = _model(dims, ranks, 10)
    y = np.random.default_rng(11).standard_normal(dims)
    g = to_dev(core, torch.float32).requires_grad_(True)
    us = [to_dev(f, torch.float32).requires_grad_(True) for f in facs]
    xh = atc.tucker_reconstruct(g, *us)
    (0.5 * ((xh - to_dev(y, torch.float32)) ** 2).sum()).backward()
    h = 1e-3
    rng = np.random.default_rng(12)

    def L(c, f):
        return 0.5 * oracle.norm2(oracle.reconstruct(c, f) - y)

    for _ in range(8):
        v = rng.standard_normal(core.shape)
        fd = (L(core + h * v, facs) - L(core - h * v, facs)) / (2 * h)
        got = float(np.sum(np64(g.grad) * v))
        assert abs(got - fd) <= 1e-4 * max(1.0, abs(fd))
    for n in range(4):
        vn = rng.standard_normal(facs[n].shape)
        fp = [f.copy() for f in facs]
        fm = [f.copy() for f in facs]
        fp[n] += h * vn
        fm[n] -= h * vn
        fd = (L(core, fp) - L(core, fm)) / (2 * h)
        got = float(np.sum(np64(us[n].grad) * vn))
        assert abs(got - fd) <= 1e-4 * max(1.0, abs(fd))
