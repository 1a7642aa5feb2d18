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


def rank_parity(t_gpu, t_orc, delta):
    """Ranks equal, or the oracle's discarded energy at the GPU rank lies within
    delta * budget of the budget (a boundary-degenerate choice)."""
    if list(t_gpu.ranks) == list(t_orc.ranks):
        return True, "exact"
    for k in range(len(t_gpu.ranks)):
        if t_gpu.ranks[k] == t_orc.ranks[k]:
            continue
        lam = t_orc.eigvals[k]
        tails = oracle.tail_sums(lam)
        b = t_orc.budgets[k]
        if abs(tails[t_gpu.ranks[k]] - b) > delta * b and abs(tails[t_orc.ranks[k]] - b) > delta * b:
            return False, "mode %d: gpu %d oracle %d" % (k, t_gpu.ranks[k], t_orc.ranks[k])
    return True, "boundary"
