"""Plain FP64 CPU oracle for the ST-HOSVD hot path (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  It shares
no code with the GPU path.  Its heavy loops (Gram matrix, mode product, one-sided
Jacobi) live in ``oracle.c``; the algorithm itself is written out here step by
step in the order of the paper.

Paper passages followed (arXiv 2107.01384):
  * Section 3.1 (tensor concepts): norm, mode-k unfolding, mode-k product;
  * Section 3.2 / Algorithm 1 (ST-HOSVD): per mode, factor from the SVD of the
    current unfolding (here: eigenvectors of its Gram matrix, whose eigenvalues
    are the squared singular values), truncation rank, projection;
  * Section 4.1.1 (mode processing order): increasing mode length by default,
    or a user order; for decompression the order minimising
    sum_i n_{p1}..n_{pi} r_{pi}..r_{pd}, found by exhaustive search;
  * Section 4.1.3 (error control): SSE target = RTMSS * target SSE, the rank of
    each mode picked dynamically inside that target, and the achieved
    truncation SSE equal to the sum of the discarded squared singular values.

Readings where the paper is silent (all listed in the design doc):
  * relative error is the norm ratio, so the SSE budget is rtmss * (eps |A|)^2;
  * rank rule 'adaptive': mode i gets (budget - used) / (modes left);
    'equal': every mode gets budget / d; r_k is the smallest r >= 1 whose
    discarded eigenvalue sum (added from the smallest up) fits the mode budget;
  * eigenvector sign: each kept column's largest-magnitude entry is positive
    (first such row on ties);
  * the core is returned in natural mode order.

Parity pins: every function here is checked by ``tests/test_oracle_*.py``
against closed forms, library routines on special cases, brute force or the
identities above.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from dataclasses import dataclass, field as dc_field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MAX_SWEEPS = 60


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no host-specific ISA)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.oracle_norm2.argtypes = [dp, i64]
    lib.oracle_norm2.restype = ctypes.c_double
    lib.oracle_gram.argtypes = [dp, i64, i64, i64, dp]
    lib.oracle_gram.restype = None
    lib.oracle_cross_gram.argtypes = [dp, i64, dp, i64, i64, i64, dp]
    lib.oracle_cross_gram.restype = None
    lib.oracle_mode_product.argtypes = [dp, i64, i64, i64, dp, i64, dp]
    lib.oracle_mode_product.restype = None
    lib.oracle_eig_jacobi.argtypes = [dp, i64, ctypes.c_int, dp, dp]
    lib.oracle_eig_jacobi.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def lnr(dims: Sequence[int], k: int):
    """(L, n, R) view of mode k of a row-major tensor of shape dims."""
    L = int(np.prod(dims[:k], dtype=np.int64))
    R = int(np.prod(dims[k + 1:], dtype=np.int64))
    return L, int(dims[k]), R


# ---------------------------------------------------------------- primitives
def norm2(x) -> float:
    """Squared Euclidean norm <X, X> (Section 3.1)."""
    x = _f64(x)
    return float(_load().oracle_norm2(_ptr(x), x.size))


def gram(y, k: int) -> np.ndarray:
    """Gram matrix Y_(k) Y_(k)^T of the mode-k unfolding (n_k x n_k)."""
    y = _f64(y)
    L, n, R = lnr(y.shape, k)
    g = np.empty((n, n))
    _load().oracle_gram(_ptr(y), L, n, R, _ptr(g))
    return g


def cross_gram(x, w, k: int) -> np.ndarray:
    """X_(k) W_(k)^T for two tensors equal in every mode but k."""
    x, w = _f64(x), _f64(w)
    L, nx, R = lnr(x.shape, k)
    L2, nw, R2 = lnr(w.shape, k)
    if (L, R) != (L2, R2):
        raise ValueError("cross_gram: tensors differ outside mode k")
    c = np.empty((nx, nw))
    _load().oracle_cross_gram(_ptr(x), nx, _ptr(w), nw, L, R, _ptr(c))
    return c


def mode_product(y, k: int, m) -> np.ndarray:
    """Z = M x_k Y, i.e. Z_(k) = M Y_(k) (Section 3.1); M has shape (m, n_k)."""
    y, m = _f64(y), _f64(m)
    L, n, R = lnr(y.shape, k)
    if m.shape[1] != n:
        raise ValueError("mode_product: matrix columns must equal n_k")
    shape = list(y.shape)
    shape[k] = m.shape[0]
    z = np.empty(shape)
    _load().oracle_mode_product(_ptr(y), L, n, R, _ptr(m), m.shape[0], _ptr(z))
    return z


def eig(g, max_sweeps: int = MAX_SWEEPS):
    """Eigenpairs of a symmetric PSD matrix by one-sided Jacobi.

    Returns (lam descending, V with eigenvectors in columns, sweeps, converged)."""
    g = _f64(g)
    n = g.shape[0]
    lam = np.empty(n)
    v = np.empty((n, n))
    s = _load().oracle_eig_jacobi(_ptr(g), n, int(max_sweeps), _ptr(lam), _ptr(v))
    return lam, v, abs(s), s > 0


# ---------------------------------------------------------------- algorithm steps
def processing_order(dims: Sequence[int], order: Optional[Sequence[int]] = None) -> List[int]:
    """Section 4.1.1: the user's order, else modes by increasing length (stable)."""
    d = len(dims)
    if order is not None:
        order = [int(k) for k in order]
        if sorted(order) != list(range(d)):
            raise ValueError("mode order must be a permutation of 0..d-1")
        return order
    return sorted(range(d), key=lambda k: (dims[k], k))


def tail_sums(lam: np.ndarray) -> np.ndarray:
    """tail[r] = sum_{j >= r} lam[j] (0-based: the energy discarded when keeping r),
    accumulated from the smallest eigenvalue upward; tail[n] = 0."""
    n = len(lam)
    tail = np.zeros(n + 1)
    acc = 0.0
    for j in range(n - 1, -1, -1):
        acc += float(lam[j])
        tail[j] = acc
    return tail


def select_rank(lam: np.ndarray, budget: float):
    """Smallest r in [1, n] whose discarded energy tail[r] fits the budget (Section 4.1.3)."""
    tail = tail_sums(lam)
    n = len(lam)
    for r in range(1, n + 1):
        if tail[r] <= budget:
            return r, float(tail[r])
    return n, 0.0  # not reached: tail[n] = 0 <= budget for budget >= 0


def sign_fix(u: np.ndarray) -> np.ndarray:
    """Make each column's largest-magnitude entry positive (first such row on ties)."""
    u = u.copy()
    for j in range(u.shape[1]):
        col = u[:, j]
        i = int(np.argmax(np.abs(col)))  # argmax returns the first maximum
        if col[i] < 0:
            u[:, j] = -col
    return u


@dataclass
class Tucker:
    core: np.ndarray
    factors: List[np.ndarray]
    ranks: List[int]
    order: List[int]
    norm2: float
    sse_pred: float
    tails: List[float]
    budgets: List[float]
    eigvals: List[np.ndarray] = dc_field(default_factory=list)
    sweeps: List[int] = dc_field(default_factory=list)
    converged: bool = True


def sthosvd(x, eps: float, order=None, rtmss: float = 1.0, rule: str = "adaptive",
            fixed_ranks: Optional[Sequence[int]] = None, max_sweeps: int = MAX_SWEEPS) -> Tucker:
    """ST-HOSVD (Algorithm 1) with Gram + eigendecomposition per mode, in FP64.

    x: array of any real dtype (converted to float64, exact for float32).
    eps: target relative error |A - A~| / |A| (Section 2.1, relative error).
    fixed_ranks: per natural mode, a rank to keep instead of the budget rule, or
    None for that mode to use the rule (the remaining budget is then shared as
    usual, so a boundary-degenerate rank of another implementation can be
    followed through the later modes).
    Returns a Tucker record: core (natural mode order), factors U_k (n_k x r_k).
    """
    if rule not in ("adaptive", "equal"):
        raise ValueError("rule must be 'adaptive' or 'equal'")
    if not (eps >= 0.0) or not (0.0 <= rtmss <= 1.0):
        raise ValueError("need eps >= 0 and 0 <= rtmss <= 1")
    y = _f64(x)
    dims = list(y.shape)
    d = len(dims)
    order = processing_order(dims, order)
    nrm2 = norm2(y)
    budget_total = rtmss * (eps * eps) * nrm2
    used = 0.0
    factors: List[Optional[np.ndarray]] = [None] * d
    ranks = list(dims)
    tails = [0.0] * d
    budgets = [0.0] * d
    eigvals: List[np.ndarray] = [None] * d  # type: ignore
    sweeps = [0] * d
    conv = True
    for i, k in enumerate(order):
        g = gram(y, k)
        lam, v, sw, ok = eig(g, max_sweeps)
        conv = conv and ok
        if rule == "adaptive":
            b = (budget_total - used) / (d - i)
        else:
            b = budget_total / d
        if fixed_ranks is not None and fixed_ranks[k] is not None:
            r = int(fixed_ranks[k])
            r_tail = float(tail_sums(lam)[r])
        else:
            r, r_tail = select_rank(lam, b)
        used += r_tail
        u = sign_fix(v[:, :r])
        y = mode_product(y, k, u.T)
        factors[k] = u
        ranks[k] = r
        tails[k] = r_tail
        budgets[k] = b
        eigvals[k] = lam
        sweeps[k] = sw
    return Tucker(core=y, factors=factors, ranks=ranks, order=order, norm2=nrm2, sse_pred=used,
                  tails=tails, budgets=budgets, eigvals=eigvals, sweeps=sweeps, converged=conv)


# ---------------------------------------------------------------- reconstruction
def reconstruct_cost(dims: Sequence[int], ranks: Sequence[int], order: Sequence[int]) -> int:
    """Section 4.1.1: sum_i n_{p1}..n_{pi} * r_{pi}..r_{pd} multiply-adds."""
    total = 0
    d = len(order)
    for i in range(d):
        t = 1
        for j in range(i + 1):
            t *= int(dims[order[j]])
        for j in range(i, d):
            t *= int(ranks[order[j]])
        total += t
    return total


def reconstruct_order(dims: Sequence[int], ranks: Sequence[int]):
    """Exhaustive search for the cheapest decompression order (first in lexicographic
    order among equal costs).  Returns (order, cost)."""
    best, best_cost = None, None
    for p in itertools.permutations(range(len(dims))):
        c = reconstruct_cost(dims, ranks, p)
        if best_cost is None or c < best_cost:
            best, best_cost = list(p), c
    return best, best_cost


def reconstruct(core, factors, order=None) -> np.ndarray:
    """(U_1, ..., U_d) . B (Section 3.2): expand every mode of the core by its factor."""
    y = _f64(core)
    dims = [f.shape[0] for f in factors]
    ranks = list(y.shape)
    if order is None:
        order, _ = reconstruct_order(dims, ranks)
    for k in order:
        y = mode_product(y, k, factors[k])
    return y


def rel_error(x, core, factors) -> float:
    """|X - X~| / |X| in FP64."""
    x = _f64(x)
    xh = reconstruct(core, factors)
    return float(np.sqrt(norm2(x - xh) / norm2(x)))


def loss_and_grad(core, factors, y):
    """L = 0.5 |X~ - Y|^2 with X~ = (U_1..U_d).G and its exact gradient in FP64.

    With D = X~ - Y: dL/dG = D x_1 U_1^T ... x_d U_d^T, and
    dL/dU_n = D_(n) W_(n)^T where W = G x_{m != n} U_m (every mode but n expanded)."""
    g = _f64(core)
    factors = [_f64(f) for f in factors]
    d = g.ndim
    xh = reconstruct(g, factors)
    dx = xh - _f64(y)
    loss = 0.5 * norm2(dx)
    dg = dx
    for k in range(d):
        dg = mode_product(dg, k, factors[k].T)
    dus = []
    for n in range(d):
        w = g
        for m in range(d):
            if m != n:
                w = mode_product(w, m, factors[m])
        dus.append(cross_gram(dx, w, n))
    return loss, dg, dus
