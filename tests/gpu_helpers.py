"""Shared helpers of the GPU parity tests (comparisons against the FP64 oracle)."""
import sys

import numpy as np
import torch

import oracle


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def np64(t):
    return t.detach().to("cpu", torch.float64).numpy()


def projector_gap(u_a, u_b):
    """max |U_a U_a^T - U_b U_b^T| (independent of signs and rotations inside the span)."""
    return float(np.abs(u_a @ u_a.T - u_b @ u_b.T).max())


def recon_rel_diff(x, t_gpu, t_orc):
    """|X~_gpu - X~_oracle| / |X| computed in FP64 by the oracle's reconstruction."""
    xg = oracle.reconstruct(np64(t_gpu.core), [np64(f) for f in t_gpu.factors])
    xo = oracle.reconstruct(t_orc.core, t_orc.factors)
    return float(np.sqrt(oracle.norm2(xg - xo) / oracle.norm2(x)))


def gpu_rel_error(x, t_gpu):
    """|X - X~_gpu| / |X| in FP64 (oracle reconstruction of the GPU core and factors)."""
    return oracle.rel_error(np.asarray(x, dtype=np.float64), np64(t_gpu.core), [np64(f) for f in t_gpu.factors])


def boundary_ok(lam, budget, r_gpu, r_orc, band):
    """A rank other than the oracle's is accepted only next to it (|r_gpu - r_orc|
    <= 1) and only when the budget cuts the spectrum where an FP32-grade Gram
    matrix cannot tell the two ranks apart.  With r1 = min(r_gpu, r_orc), the
    two runs disagree on one comparison only: whether the discarded energy at
    r1 fits the budget.  The oracle's discarded energy at r1 must therefore lie
    within band * budget of the budget (from below when the GPU kept one more
    vector, from above when it kept one fewer)."""
    if abs(r_gpu - r_orc) > 1:
        return False
    tails = oracle.tail_sums(lam)
    r1 = min(r_gpu, r_orc)
    return abs(tails[r1] - budget) <= band * budget


def rank_parity(x, t_gpu, t_orc, band, eps, **oracle_kw):
    """Ranks equal to the oracle's, or boundary-degenerate mode by mode.

    Modes are walked in processing order.  At a mode whose GPU rank differs,
    boundary_ok must hold against the oracle run that has followed the GPU's
    ranks so far; the oracle is then re-run with the GPU's ranks fixed on the
    modes processed up to here (budget rule on the rest), so the later modes
    are judged on the tensor and remaining budget the GPU actually had.
    Returns (ok, how, oracle record that followed the GPU's ranks)."""
    if list(t_gpu.ranks) == list(t_orc.ranks):
        return True, "exact", t_orc
    d = len(t_gpu.ranks)
    t = t_orc
    fixed = [None] * d
    for i, k in enumerate(t_orc.order):
        if t_gpu.ranks[k] != t.ranks[k]:
            if not boundary_ok(t.eigvals[k], t.budgets[k], t_gpu.ranks[k], t.ranks[k], band):
                tails = oracle.tail_sums(t.eigvals[k])
                r1 = min(t_gpu.ranks[k], t.ranks[k])
                return False, "mode %d: gpu %d oracle %d (oracle tail at rank %d / budget = %.4f)" % (
                    k, t_gpu.ranks[k], t.ranks[k], r1, tails[r1] / t.budgets[k]), t
            for j in t_orc.order[: i + 1]:
                fixed[j] = t_gpu.ranks[j]
            t = oracle.sthosvd(x, eps, fixed_ranks=fixed, **oracle_kw)
    return True, "boundary", t


def rank_misses(t_gpu, t_orc):
    return sum(int(a != b) for a, b in zip(t_gpu.ranks, t_orc.ranks))
