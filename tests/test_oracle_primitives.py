"""Pins for the oracle's primitives (CPU only).

Each primitive is checked against something other than itself: a different
route through numpy (explicit unfolding by moveaxis/reshape and a matrix
product, einsum), a library eigensolver (LAPACK through numpy.linalg.eigh),
brute-force Python loops on tiny inputs, and identities (trace, symmetry,
positive semidefiniteness, orthogonality).
"""
import itertools

import numpy as np
import pytest

import oracle

SHAPES = [(5, 6, 7), (1, 9, 4), (7, 1, 3), (3, 4, 1), (2, 3, 4, 5), (13,), (4, 4)]


def unfold(x, k):
    """Mode-k matricization (Section 3.1): mode-k fibers as columns."""
    return np.moveaxis(x, k, 0).reshape(x.shape[k], -1)


@pytest.mark.parametrize("shape", SHAPES)
def test_gram_matches_unfolding_product(shape):
    rng = np.random.default_rng(11)
    x = rng.standard_normal(shape)
    for k in range(len(shape)):
        g = oracle.gram(x, k)
        xu = unfold(x, k)
        ref = xu @ xu.T
        assert np.allclose(g, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
        assert np.array_equal(g, g.T)
        assert abs(np.trace(g) - np.sum(x * x)) <= 1e-13 * np.sum(x * x)
        assert np.linalg.eigvalsh(g).min() >= -1e-12 * max(1.0, np.abs(g).max())


def test_gram_brute_force_tiny():
    rng = np.random.default_rng(12)
    x = rng.standard_normal((3, 4, 2))
    k = 1
    g = oracle.gram(x, k)
    for a, b in itertools.product(range(4), range(4)):
        s = 0.0
        for i0 in range(3):
            for i2 in range(2):
                s += x[i0, a, i2] * x[i0, b, i2]
        assert abs(g[a, b] - s) <= 1e-14 * max(1.0, abs(s))


@pytest.mark.parametrize("shape", SHAPES)
def test_mode_product_matches_einsum(shape):
    rng = np.random.default_rng(13)
    x = rng.standard_normal(shape)
    letters = "abcdefgh"[: len(shape)]
    for k in range(len(shape)):
        m = rng.standard_normal((3, shape[k]))
        z = oracle.mode_product(x, k, m)
        out = letters[:k] + "z" + letters[k + 1:]
        ref = np.einsum("z" + letters[k] + "," + letters + "->" + out, m, x)
        assert z.shape == ref.shape
        assert np.allclose(z, ref, rtol=1e-13, atol=1e-13)


def test_mode_product_properties():
    """Section 3.1: products along different modes commute; along one mode they compose;
    an orthogonal matrix preserves the norm."""
    rng = np.random.default_rng(14)
    x = rng.standard_normal((4, 5, 6))
    a = rng.standard_normal((3, 4))
    b = rng.standard_normal((2, 6))
    ab = oracle.mode_product(oracle.mode_product(x, 0, a), 2, b)
    ba = oracle.mode_product(oracle.mode_product(x, 2, b), 0, a)
    assert np.allclose(ab, ba, rtol=1e-13, atol=1e-13)
    c = rng.standard_normal((7, 3))
    comp = oracle.mode_product(oracle.mode_product(x, 0, a), 0, c)
    assert np.allclose(comp, oracle.mode_product(x, 0, c @ a), rtol=1e-12, atol=1e-12)
    q, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    assert np.isclose(oracle.norm2(oracle.mode_product(x, 1, q)), oracle.norm2(x), rtol=1e-13)


def test_cross_gram_matches_unfolding_product():
    rng = np.random.default_rng(15)
    x = rng.standard_normal((3, 5, 4))
    w = rng.standard_normal((3, 2, 4))
    c = oracle.cross_gram(x, w, 1)
    assert np.allclose(c, unfold(x, 1) @ unfold(w, 1).T, rtol=1e-13, atol=1e-13)


def test_norm2():
    rng = np.random.default_rng(16)
    x = rng.standard_normal(100003)
    assert abs(oracle.norm2(x) - float(np.dot(x, x))) <= 1e-12 * float(np.dot(x, x))
    assert oracle.norm2(np.zeros(7)) == 0.0
    assert oracle.norm2(np.array([3.0, 4.0])) == 25.0


def _check_eig(g, tol=1e-12):
    lam, v, sweeps, ok = oracle.eig(g)
    n = g.shape[0]
    assert ok
    ref = np.sort(np.linalg.eigvalsh(g))[::-1]
    scale = max(np.abs(g).max(), 1e-300)
    assert np.all(np.diff(lam) <= 0)
    assert np.allclose(lam, np.clip(ref, 0, None), rtol=0, atol=tol * n * scale)
    assert np.allclose(v.T @ v, np.eye(n), atol=tol * n)
    assert np.abs(g @ v - v * lam).max() <= tol * n * scale
    return lam, v


@pytest.mark.parametrize("n", [1, 2, 3, 8, 33, 64, 97])
def test_eig_random_psd(n):
    rng = np.random.default_rng(17 + n)
    a = rng.standard_normal((n, 2 * n + 3))
    _check_eig(a @ a.T)


def test_eig_graded_spectrum():
    """Eigenvalues over 12 orders of magnitude (like a smooth field's Gram matrix)."""
    rng = np.random.default_rng(18)
    n = 40
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam_true = np.logspace(0, -12, n)
    g = (q * lam_true) @ q.T
    g = 0.5 * (g + g.T)
    lam, v = _check_eig(g)
    assert np.allclose(lam[:10], lam_true[:10], rtol=1e-10)


def test_eig_degenerate_and_special():
    # exactly repeated eigenvalues
    rng = np.random.default_rng(19)
    q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    g = (q * np.array([5.0, 5.0, 5.0, 1.0, 1.0, 0.0])) @ q.T
    g = 0.5 * (g + g.T)
    lam, v = _check_eig(g)
    # the 3-dimensional eigenspace is reproduced as a subspace
    p_ref = q[:, :3] @ q[:, :3].T
    p = v[:, :3] @ v[:, :3].T
    assert np.abs(p - p_ref).max() < 1e-12
    # diagonal input: exact eigenvalues, unit eigenvectors, order by value then index
    lam, v, _, ok = oracle.eig(np.diag([1.0, 4.0, 4.0, 2.0]))
    assert ok and list(lam) == [4.0, 4.0, 2.0, 1.0]
    assert np.array_equal(np.abs(v), np.eye(4)[:, [1, 2, 3, 0]])
    # zero matrix
    lam, v, _, ok = oracle.eig(np.zeros((5, 5)))
    assert ok and np.all(lam == 0) and np.array_equal(v, np.eye(5))


def test_eig_sweep_cap_reports_nonconvergence():
    rng = np.random.default_rng(20)
    a = rng.standard_normal((20, 30))
    lam, v, sweeps, ok = oracle.eig(a @ a.T, max_sweeps=1)
    assert not ok and sweeps == 1
