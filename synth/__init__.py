"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and evaluates the closed-form test fields;
it contains none of the ST-HOSVD arithmetic (no Gram, eigensolver, rank choice or
mode product of the method).  Every generator is deterministic in its seed.

Stand-ins for the paper's datasets (Section 6.1, Table 4): the paper's volumes
(Isotropic turbulence, Hurricane, ...) are not available here, so smooth
multi-scale fields of the same shapes are built from Gaussian blobs, plane waves
and white noise.

Field F(shape, seed) for a 3-D shape (n0, n1, n2):
  * grid x_a = (i + 0.5) / n_a on the unit cube, per axis a;
  * 32 blobs; blob b draws centre c = U[0,1]^3 and then widths s = U[0.02, 0.2]^3,
    and adds prod_a exp(-(x_a - c_a)^2 / (2 s_a^2)) with amplitude 1;
  * 8 plane waves; wave w draws integer k in {-4..4}^3 and then phase phi in
    U[0, 2 pi), and adds sin(2 pi k . x + phi);
  * white noise 1e-4 * N(0, 1) over the whole grid (C order);
  * evaluated in float64 and returned as float32 (or float64 when asked).

Both the blobs and the waves are sums of separable terms (sin(a+b+c) expands into
four products), so the smooth part is evaluated as one small matrix product of
per-axis profiles; the result equals the pointwise formula up to float64 rounding.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "field",
    "field4",
    "tucker_c1",
    "known_rank_tucker",
    "batch_dims",
    "batch_arena",
    "recon_model",
    "BLOCK_SIZES",
]

N_BLOBS = 32
N_WAVES = 8
NOISE_STD = 1e-4
BLOCK_SIZES = (16, 24, 32, 48, 64)


def _axis_grid(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def _field_profiles(shape, rng):
    """Per-axis profiles (T, n_a) of the separable smooth part, in draw order."""
    xs = [_axis_grid(n) for n in shape]
    prof = [[] for _ in range(3)]
    for _ in range(N_BLOBS):
        c = rng.uniform(0.0, 1.0, 3)
        s = rng.uniform(0.02, 0.2, 3)
        for a in range(3):
            prof[a].append(np.exp(-((xs[a] - c[a]) ** 2) / (2.0 * s[a] ** 2)))
    for _ in range(N_WAVES):
        k = rng.integers(-4, 5, 3)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        # angle per axis; the phase rides on axis 0
        th = [2.0 * np.pi * k[a] * xs[a] for a in range(3)]
        th[0] = th[0] + phi
        sa, ca = np.sin(th[0]), np.cos(th[0])
        sb, cb = np.sin(th[1]), np.cos(th[1])
        sc, cc = np.sin(th[2]), np.cos(th[2])
        # sin(a+b+c) = sa cb cc + ca sb cc + ca cb sc - sa sb sc
        for p0, p1, p2 in ((sa, cb, cc), (ca, sb, cc), (ca, cb, sc), (-sa, sb, sc)):
            prof[0].append(p0)
            prof[1].append(p1)
            prof[2].append(p2)
    return [np.stack(p) for p in prof]  # each (T, n_a)


def field(shape, seed: int, dtype=np.float32, noise_std: float = NOISE_STD) -> np.ndarray:
    """Smooth 3-D test field F(shape, seed) (see module docstring)."""
    shape = tuple(int(n) for n in shape)
    if len(shape) != 3:
        raise ValueError("field() builds 3-D fields")
    rng = np.random.default_rng(seed)
    P0, P1, P2 = _field_profiles(shape, rng)
    n0, n1, n2 = shape
    out = np.empty(shape, dtype=dtype)
    # slabs along axis 0 keep the float64 temporaries small; the noise is drawn in
    # C order slab by slab, which reproduces one standard_normal(shape) draw.
    slab = max(1, min(n0, (1 << 24) // max(1, n1 * n2)))
    for i0 in range(0, n0, slab):
        i1 = min(n0, i0 + slab)
        kr = (P0[:, i0:i1, None] * P1[:, None, :]).reshape(P0.shape[0], -1)  # (T, s*n1)
        smooth = (kr.T @ P2).reshape(i1 - i0, n1, n2)
        if noise_std:
            smooth += noise_std * rng.standard_normal((i1 - i0, n1, n2))
        out[i0:i1] = smooth
    return out


def field4(shape3=(200, 500, 500), nvar: int = 13, seed0: int = 100, dtype=np.float32) -> np.ndarray:
    """4-way variant: nvar independent fields F(shape3, seed0 + f) stacked on the last mode."""
    out = np.empty(tuple(shape3) + (nvar,), dtype=dtype)
    for f in range(nvar):
        out[..., f] = field(shape3, seed0 + f, dtype=dtype)
    return out


def _qr_q(rng, n: int, r: int) -> np.ndarray:
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def _mode_apply(t: np.ndarray, k: int, m: np.ndarray) -> np.ndarray:
    """Multiply mode k of t by the matrix m (rows of m index the new mode)."""
    return np.moveaxis(np.tensordot(m, t, axes=([1], [k])), 0, k)


def known_rank_tucker(dims, ranks, seed: int, rel_noise: float = 0.0):
    """Tensor of exact multilinear rank `ranks` (iid N(0,1) core, orthonormal factors
    from QR of Gaussians), optionally plus iid noise of std rel_noise * rms.

    Returns (x float64, core, factors)."""
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(tuple(ranks))
    facs = [_qr_q(rng, n, r) for n, r in zip(dims, ranks)]
    t = core
    for k, u in enumerate(facs):
        t = _mode_apply(t, k, u)
    if rel_noise:
        rms = np.sqrt(np.mean(t * t))
        t = t + rel_noise * rms * rng.standard_normal(t.shape)
    return np.ascontiguousarray(t), core, facs


def tucker_c1(noise: str = "relative"):
    """64^3 float64 known-rank-8 Tucker tensor plus noise (seed 1).

    noise='relative': std 1e-3 * rms(T) (the reading that gives ranks 8,8,8);
    noise='absolute': std 1e-3; noise='none': noiseless."""
    rng = np.random.default_rng(1)
    core = rng.standard_normal((8, 8, 8))
    facs = [_qr_q(rng, 64, 8) for _ in range(3)]
    t = core
    for k, u in enumerate(facs):
        t = _mode_apply(t, k, u)
    if noise == "relative":
        t = t + 1e-3 * np.sqrt(np.mean(t * t)) * rng.standard_normal(t.shape)
    elif noise == "absolute":
        t = t + 1e-3 * rng.standard_normal(t.shape)
    elif noise != "none":
        raise ValueError(noise)
    return np.ascontiguousarray(t)


def batch_dims(nblocks: int = 4096, seed: int = 2024) -> np.ndarray:
    """(nblocks, 3) int32 block shapes drawn uniformly from BLOCK_SIZES per mode."""
    rng = np.random.default_rng(seed)
    return rng.choice(np.array(BLOCK_SIZES, dtype=np.int32), size=(nblocks, 3)).astype(np.int32)


def batch_arena(dims: np.ndarray, seed0: int = 10_000, dtype=np.float32):
    """Pack block b = F(dims[b], seed0 + b) contiguously; returns (arena, offsets int64)."""
    sizes = np.prod(dims.astype(np.int64), axis=1)
    offsets = np.zeros(len(dims), dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)[:-1]
    arena = np.empty(int(sizes.sum()), dtype=dtype)
    for b, d in enumerate(dims):
        arena[offsets[b]: offsets[b] + sizes[b]] = field(tuple(d), seed0 + b, dtype=dtype).ravel()
    return arena, offsets


def recon_model(dims=(128, 128, 128, 64), ranks=(32, 32, 32, 16), seed: int = 3, with_target: bool = True,
                target_seed0: int = 300):
    """Tucker model for the differentiable reconstruction: core iid N(0,1), factors from QR
    of Gaussians (seed 3); target Y stacks dims[3] fields F(dims[:3], target_seed0 + j)."""
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(tuple(ranks))
    facs = [_qr_q(rng, n, r) for n, r in zip(dims, ranks)]
    y = None
    if with_target:
        y = np.empty(tuple(dims), dtype=np.float32)
        for j in range(dims[3]):
            y[..., j] = field(tuple(dims[:3]), target_seed0 + j)
    return core, facs, y
