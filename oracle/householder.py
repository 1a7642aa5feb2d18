"""Plain FP64 CPU oracle of the Householder factor representation and of the
hybrid error model (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the GPU library or
its binding; it shares no code with the GPU path.

Paper passages followed (arXiv 2107.01384):
  * Supplement S.2 (Householder-based factor compression, its algorithm): a
    factor U (n x r, orthonormal columns) is written as the product of r
    Householder reflectors H_j = I - 2 v_j v_j^T, v_j of unit norm and zero
    above row j; the reflectors come from Householder QR of U, column by
    column, and the columns of U whose R_jj came out negative are flipped, so
    that U' = H_1 ... H_r [I_r; 0] exactly.  v_jj is the largest entry of v_j
    in magnitude and is not stored (it follows from |v_j| = 1): n r - r(r+1)/2
    coefficients remain.
  * Supplement S.2 (weights): before quantization the entries of v_j are
    scaled by sqrt(2 alpha_j), alpha_j from the slice norms sigma of the
    quantized core and n_j = n - j + 1 (j 1-based).
  * Section 4.1.3, eq. (total_error_approximation): the squared compression
    error is predicted as the ST-HOSVD's discarded energy, plus the core's
    quantization error, plus sum_i |dU_i Sigma_i|_F^2, Sigma_i the mode-i
    slice norms of the quantized core.

Readings (listed in the design doc):
  * sgn(0) = +1 when forming v_j;
  * v_j is stored with v_jj > 0 (H_j does not change when v_j changes sign),
    and decoding takes v_jj = sqrt(max(0, 1 - sum_{i>j} v_ij^2));
  * the coefficients are laid out column by column (column j: rows j+1 .. n-1);
  * alpha_j's second term is taken as zero when no column follows j (its
    factor 2/(n_j - 1) is then undefined for n_j = 1 but multiplies an empty
    sum).
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np


def reflectors(U) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(V, signs, U') of a factor with orthonormal columns: V (n x r) holds v_j
    in column j (zero above row j, v_jj > 0), signs[j] = sgn(R_jj) of the
    Householder QR, U' = U diag(signs) (supplement S.2)."""
    R = np.array(U, dtype=np.float64, copy=True)
    n, r = R.shape
    V = np.zeros((n, r))
    signs = np.ones(r)
    for j in range(r):
        x = R[j:, j].copy()
        nx = math.sqrt(float(np.dot(x, x)))
        v = x.copy()
        v[0] += (1.0 if x[0] >= 0.0 else -1.0) * nx
        nv = math.sqrt(float(np.dot(v, v)))
        if nv == 0.0:             # a zero column: nothing to reflect
            v = np.zeros_like(x)
            v[0] = 1.0
        else:
            v /= nv
        # apply H_j = I - 2 v v^T to the trailing block
        R[j:, j:] -= 2.0 * np.outer(v, v @ R[j:, j:])
        signs[j] = 1.0 if R[j, j] >= 0.0 else -1.0
        if v[0] < 0.0:
            v = -v
        V[j:, j] = v
    return V, signs, np.asarray(U, dtype=np.float64) * signs


def ncoef(n: int, r: int) -> int:
    return n * r - r * (r + 1) // 2


def coefficients(V) -> np.ndarray:
    """The stored entries: column by column, the rows below the diagonal."""
    n, r = V.shape
    return np.concatenate([V[j + 1:, j] for j in range(r)]) if r else np.zeros(0)


def from_coefficients(c, n: int, r: int) -> np.ndarray:
    """V from the stored entries, v_jj = sqrt(max(0, 1 - sum_{i>j} v_ij^2))."""
    V = np.zeros((n, r))
    pos = 0
    for j in range(r):
        m = n - j - 1
        V[j + 1:, j] = c[pos: pos + m]
        pos += m
        V[j, j] = math.sqrt(max(0.0, 1.0 - float(np.dot(V[j + 1:, j], V[j + 1:, j]))))
    return V


def factor(V, r: int) -> np.ndarray:
    """U' = H_1 H_2 ... H_r applied to the first r columns of the identity."""
    n = V.shape[0]
    X = np.zeros((n, r))
    X[:r, :r] = np.eye(r)
    for j in range(r - 1, -1, -1):
        v = V[:, j]
        X -= 2.0 * np.outer(v, v @ X)
    return X


def alpha(sigma: Sequence[float], n: int) -> np.ndarray:
    """alpha_j of supplement S.2 for a factor with n rows and the slice norms
    sigma_1 .. sigma_r of the quantized core in its mode."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    r = s2.size
    a = np.zeros(r)
    for j in range(1, r + 1):
        nj = n - j + 1
        rt = math.sqrt(nj)
        own = (1.0 + (nj + 5.0 * rt + 2.0) / ((rt + 1.0) ** 2 * rt)) * s2[j - 1]
        rest = float(np.sum(s2[j:]))
        later = 0.0
        if j < r:
            later = (2.0 / (nj - 1) + (nj + 2.0 * rt + 2.0) / ((rt + 1.0) ** 3 * rt)) * rest
        a[j - 1] = own + later
    return a


def coefficient_weights(sigma, n: int) -> np.ndarray:
    """sqrt(2 alpha_j) repeated over the stored entries of column j."""
    a = alpha(sigma, n)
    r = a.size
    return np.concatenate([np.full(n - j - 1, math.sqrt(2.0 * a[j])) for j in range(r)]) if r else np.zeros(0)


def slice_norms2(core) -> list:
    """Per mode i, the squared norms of the mode-i slices of the core."""
    c = np.asarray(core, dtype=np.float64)
    out = []
    for k in range(c.ndim):
        axes = tuple(a for a in range(c.ndim) if a != k)
        out.append(np.sum(c * c, axis=axes))
    return out


def factor_error_term(U, Uq, sigma2) -> float:
    """|dU Sigma|_F^2 = sum_j sigma_j^2 |Uq[:, j] - U[:, j]|^2 (eq. total_error_approximation)."""
    d = np.asarray(Uq, dtype=np.float64) - np.asarray(U, dtype=np.float64)
    return float(np.sum(np.sum(d * d, axis=0) * np.asarray(sigma2, dtype=np.float64)))


def predicted_error(sthosvd_sse: float, core_sse: float, factor_terms: Sequence[float]) -> float:
    """Eq. (total_error_approximation): the three error components added."""
    return float(sthosvd_sse) + float(core_sse) + float(sum(factor_terms))


def encode(U, sigma2=None):
    """(weighted coefficients, signs, U') of a factor: the reflectors' stored
    entries, each column's scaled by sqrt(2 alpha_j) when the core's squared
    slice norms are given (supplement S.2)."""
    V, signs, Up = reflectors(U)
    n, r = V.shape
    c = coefficients(V)
    if sigma2 is not None:
        c = c * coefficient_weights(np.sqrt(np.asarray(sigma2, dtype=np.float64)), n)
    return c, signs, Up


def decode(c, n: int, r: int, sigma2=None) -> np.ndarray:
    """The factor U' from (weighted) stored entries.  A zero weight only occurs
    once every later slice norm is zero as well; such columns multiply nothing
    and decode with v_j = e_j."""
    c = np.asarray(c, dtype=np.float64)
    if sigma2 is not None:
        w = coefficient_weights(np.sqrt(np.asarray(sigma2, dtype=np.float64)), n)
        c = np.divide(c, w, out=np.zeros_like(c), where=w > 0)
    return factor(from_coefficients(c, n, r), r)
