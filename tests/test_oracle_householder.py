"""Pins of the Householder factor representation and of the error model terms
(oracle/householder.py), against what the paper, LAPACK and the algebra fix:

* the representation is exact: H_1 ... H_r [I; 0] rebuilds the sign-adjusted
  factor (supplement S.2), which differs from the factor by column signs only;
* LAPACK's Householder QR (numpy.linalg.qr, mode 'raw' = dgeqrf) gives the same
  reflectors once normalised, and its R's diagonal gives the same signs;
* n r - r (r + 1) / 2 stored entries, v_jj the largest entry of v_j;
* the weights alpha_j of supplement S.2 against two values worked by hand, and
  against the first-order sensitivity they are derived from: perturbing the
  stored entries of v_j by delta grows |dU Sigma|_F^2 by 2 alpha_j delta^2
  (measured by rebuilding the factor; a wrong exponent or sign in the
  transcription moves the ratio far from 1);
* the error model (eq. total_error_approximation): with exact factors the
  squared error is exactly the truncation error plus the core's quantization
  error; for a core whose mode-i slices are orthogonal, |dU_i x_i B|^2 equals
  |dU_i Sigma_i|_F^2 exactly.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import householder as hh


def _orth(n, r, seed):
    rng = np.random.default_rng(seed)
    return np.linalg.qr(rng.standard_normal((n, r)))[0]


@pytest.mark.parametrize("n,r", [(1, 1), (5, 1), (6, 6), (64, 8), (200, 20), (512, 18), (33, 31)])
def test_representation_is_exact(n, r):
    U = _orth(n, r, n + r)
    V, s, Up = hh.reflectors(U)
    assert np.all(np.abs(s) == 1.0)
    assert np.allclose(Up, U * s, atol=0, rtol=0)
    assert np.abs(hh.factor(V, r) - Up).max() <= 1e-14 * max(1, r)
    # v_j: unit norm, zero above row j, v_jj > 0 and the largest in magnitude
    for j in range(r):
        v = V[:, j]
        assert abs(np.dot(v, v) - 1.0) <= 1e-14
        assert np.all(v[:j] == 0.0)
        assert v[j] > 0 and v[j] >= np.abs(v[j + 1:]).max(initial=0.0)
    c = hh.coefficients(V)
    assert c.size == hh.ncoef(n, r) == n * r - r * (r + 1) // 2
    assert np.abs(hh.from_coefficients(c, n, r) - V).max() <= 1e-15
    assert np.abs(hh.decode(*hh.encode(U)[:1], n, r) - Up).max() <= 1e-14 * max(1, r)


@pytest.mark.parametrize("n,r", [(7, 3), (64, 8), (300, 25)])
def test_reflectors_match_lapack_geqrf(n, r):
    U = _orth(n, r, 3 * n + r)
    V, s, _ = hh.reflectors(U)
    h, tau = np.linalg.qr(U, mode="raw")
    h = h.T  # row-major view: R above the diagonal, reflector tails below
    for j in range(r):
        w = np.zeros(n)
        w[j] = 1.0
        w[j + 1:] = h[j + 1:, j]
        if tau[j] == 0.0:
            continue
        # H = I - tau w w^T with tau = 2 / |w|^2 for a reflector
        assert abs(tau[j] - 2.0 / np.dot(w, w)) <= 1e-12
        assert np.abs(w / np.linalg.norm(w) - V[:, j]).max() <= 1e-12
        assert np.sign(h[j, j]) == s[j]


def test_alpha_hand_values():
    # n = 4, sigma = (2, 1).  j = 1: n_1 = 4, sqrt = 2:
    #   (1 + (4 + 10 + 2) / (3^2 * 2)) * 4 + (2/3 + (4 + 4 + 2) / (3^3 * 2)) * 1
    #   = (1 + 16/18) * 4 + 2/3 + 10/54 = 68/9 + 46/54 = 8.407407407...
    # j = 2: n_2 = 3, sqrt(3) = 1.7320508075688772:
    #   1 + (5 + 5 sqrt 3) / ((sqrt 3 + 1)^2 sqrt 3) = 1 + 13.660254037844386 / 12.928203230275509
    #   = 2.0566243270259355 (no later columns)
    a = hh.alpha([2.0, 1.0], 4)
    assert abs(a[0] - (68.0 / 9.0 + 46.0 / 54.0)) <= 1e-12
    assert abs(a[1] - 2.0566243270259355) <= 1e-12


@pytest.mark.parametrize("n,r,seed", [(64, 8, 0), (200, 20, 1), (512, 18, 2)])
def test_alpha_is_the_first_order_sensitivity(n, r, seed):
    rng = np.random.default_rng(seed)
    U = _orth(n, r, seed)
    V, s, Up = hh.reflectors(U)
    sig = np.sort(rng.uniform(0.1, 10.0, r))[::-1]
    a = hh.alpha(sig, n)
    meas = pred = 0.0
    for j in range(r):
        for _ in range(8):
            d = 1e-6 * rng.standard_normal(n - j - 1)
            V2 = V.copy()
            V2[j + 1:, j] += d
            V2[j, j] = math.sqrt(max(0.0, 1.0 - float(np.dot(V2[j + 1:, j], V2[j + 1:, j]))))
            dU = hh.factor(V2, r) - Up
            meas += float(np.sum((dU * sig) ** 2))
            pred += 2.0 * a[j] * float(np.dot(d, d))
    assert 0.9 <= meas / pred <= 1.1, meas / pred


def test_error_model_exact_with_exact_factors():
    """Orthonormal factors: |A - (U).B~|^2 = |A - (U).B|^2 + |B~ - B|^2."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((12, 10, 9)) * np.logspace(0, -2, 9)
    t = oracle.sthosvd(x, 1e-1)
    dB = 1e-3 * rng.standard_normal(t.core.shape)
    e_trunc = oracle.norm2(x - oracle.reconstruct(t.core, t.factors))
    e_tot = oracle.norm2(x - oracle.reconstruct(t.core + dB, t.factors))
    pred = hh.predicted_error(e_trunc, oracle.norm2(dB), [0.0, 0.0, 0.0])
    assert abs(e_tot - pred) <= 1e-10 * e_tot


def test_factor_term_exact_for_orthogonal_slices():
    """A core whose mode-0 slices are orthogonal (a diagonal core):
    |dU x_0 B|^2 = |dU Sigma|_F^2 exactly."""
    rng = np.random.default_rng(5)
    r = 6
    B = np.zeros((r, r, r))
    for i in range(r):
        B[i, i, i] = 10.0 / (i + 1)
    dU = 1e-3 * rng.standard_normal((20, r))
    lhs = oracle.norm2(oracle.mode_product(B, 0, dU))
    s2 = hh.slice_norms2(B)[0]
    assert abs(lhs - hh.factor_error_term(np.zeros((20, r)), dU, s2)) <= 1e-12 * lhs
