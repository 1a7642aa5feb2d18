"""GPU parity of atc_sthosvd against the FP64 oracle (called through the C ABI).

Bars:
  * FP64 path: ranks identical, predicted SSE within 1e-9 relative, kept
    subspaces (projectors) within 1e-9, reconstruction within 1e-11 of the
    oracle's (relative to |X|).
  * FP32 and BF16X3 paths: ranks identical or boundary-degenerate (the oracle's
    discarded energy at the smaller of the two ranks within 10% of the mode budget), achieved
    error <= 1.02 eps, and |X~_gpu - X~_oracle| / |X| reported and bounded.
Shapes cover every loader layout of the Gram and mode-product kernels
(contiguous-R, R == 1, 1 < R < tile depth), ragged tiles (n not a multiple
of 64) and both eigensolver paths (dense Jacobi, subspace iteration).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2107_01384_amd as atc
import synth
from gpu_helpers import gpu_rel_error, log, np64, projector_gap, rank_parity, recon_rel_diff, to_dev

pytestmark = pytest.mark.gpu


def _run(x, eps, dtype, **kw):
    log("sthosvd", x.shape, dtype, eps, kw)
    xd = to_dev(x, dtype)
    t = atc.sthosvd(xd, eps, **kw)
    torch.cuda.synchronize()
    return t


def _eigvec_tol(lam, r):
    """Entry-wise bound for the kept eigenvectors of an FP64 Gram matrix: a
    perturbation of size ~n u |G| moves eigenvector j by about that over its gap
    to the neighbouring eigenvalues."""
    lam = np.asarray(lam, dtype=np.float64)
    n = len(lam)
    gaps = []
    for j in range(r):
        g = np.inf
        if j > 0:
            g = min(g, lam[j - 1] - lam[j])
        if j + 1 < n:
            g = min(g, lam[j] - lam[j + 1])
        gaps.append(g)
    gap = max(min(gaps), 1e-300)
    return min(1e-2, 64 * n * 2.0 ** -53 * lam[0] / gap)


F64_SHAPES = [(5, 6, 7), (13, 17, 3), (70, 9, 11), (3, 130, 20), (40, 33, 2, 5), (257,), (12, 40)]


@pytest.mark.parametrize("shape", F64_SHAPES)
def test_f64_parity_random(shape):
    rng = np.random.default_rng(sum(shape))
    # graded spectrum so that the budget cuts at a well separated point
    x = rng.standard_normal(shape)
    for k, n in enumerate(shape):
        scale = np.logspace(0, -3, n).reshape([-1 if i == k else 1 for i in range(len(shape))])
        x = x * scale
    for eps in (1e-1, 1e-2):
        t_o = oracle.sthosvd(x, eps)
        t_g = _run(x, eps, torch.float64)
        assert t_g.ranks == t_o.ranks, (t_g.ranks, t_o.ranks)
        assert t_g.order == t_o.order
        assert abs(t_g.norm2 - t_o.norm2) <= 1e-12 * t_o.norm2
        assert abs(t_g.sse_pred - t_o.sse_pred) <= 1e-9 * t_o.norm2
        tol_u = 0.0
        for k in range(len(shape)):
            assert projector_gap(np64(t_g.factors[k]), t_o.factors[k]) < 1e-9
            # the sign rule is applied on both sides: factors agree entry by entry,
            # to the eigenvector accuracy that the kept eigenvalues' gaps allow
            tol = _eigvec_tol(t_o.eigvals[k], t_o.ranks[k])
            tol_u = max(tol_u, tol)
            du = np.abs(np64(t_g.factors[k]) - t_o.factors[k]).max()
            assert du <= tol, (k, du, tol)
        # the core follows from the factors: entry by entry as well
        dc = np.abs(np64(t_g.core) - t_o.core).max()
        assert dc <= len(shape) * tol_u * np.sqrt(t_o.norm2) + 1e-13 * np.sqrt(t_o.norm2), (dc, tol_u)
        assert recon_rel_diff(x, t_g, t_o) < 1e-11
        assert gpu_rel_error(x, t_g) <= eps * (1 + 1e-9)


def test_f64_config_64cube_known_rank():
    """64^3 float64 Tucker (core 8^3) + 1e-3 relative noise at eps = 1e-2: ranks (8,8,8)."""
    x = synth.tucker_c1("relative")
    t_o = oracle.sthosvd(x, 1e-2, order=[0, 1, 2])
    t_g = _run(x, 1e-2, torch.float64, order=[0, 1, 2])
    assert t_g.ranks == [8, 8, 8] == t_o.ranks
    err = gpu_rel_error(x, t_g)
    assert err <= 1.02e-2
    assert abs(err - oracle.rel_error(x, t_o.core, t_o.factors)) <= 1e-12
    for k in range(3):
        assert projector_gap(np64(t_g.factors[k]), t_o.factors[k]) < 1e-10
        tol = _eigvec_tol(t_o.eigvals[k], 8)
        assert np.abs(np64(t_g.factors[k]) - t_o.factors[k]).max() <= tol, k
    assert np.abs(np64(t_g.core) - t_o.core).max() <= 1e-9 * np.abs(t_o.core).max()
    log("C1 ranks", t_g.ranks, "err", err)


def test_f64_noiseless_exact_recovery():
    x, core, facs = synth.known_rank_tucker((48, 40, 56), (4, 6, 5), seed=3)
    t_g = _run(x, 1e-6, torch.float64)
    assert t_g.ranks == [4, 6, 5]
    assert gpu_rel_error(x, t_g) < 1e-13
    for k in range(3):
        assert projector_gap(np64(t_g.factors[k]), facs[k]) < 1e-12


def test_f64_fixed_ranks_and_equal_rule():
    x = synth.field((20, 24, 28), 4).astype(np.float64)
    t_o = oracle.sthosvd(x, 1e-2, fixed_ranks=[3, 5, 7])
    t_g = _run(x, 1e-2, torch.float64, fixed_ranks=[3, 5, 7])
    assert t_g.ranks == [3, 5, 7]
    assert abs(t_g.sse_pred - t_o.sse_pred) <= 1e-9 * t_o.norm2
    t_o = oracle.sthosvd(x, 1e-3, rule="equal")
    t_g = _run(x, 1e-3, torch.float64, rule="equal")
    assert t_g.ranks == t_o.ranks
    assert recon_rel_diff(x, t_g, t_o) < 1e-11


# (shape, eps): layouts: mode-0 contiguous R, middle modes R == 13 (1 < R < 32),
# last mode R == 1; n = 70, 100 > 64 use the subspace eigensolver
F32_CASES = [((24, 36, 40), 1e-2), ((33, 64, 13), 1e-3), ((48, 20, 29, 13), 1e-3), ((100, 70, 45), 1e-3),
             ((16, 16, 16), 1e-4)]


@pytest.mark.parametrize("precision", ["native", "bf16x3", "f64acc"])
@pytest.mark.parametrize("shape,eps", F32_CASES)
def test_f32_parity_fields(shape, eps, precision):
    if len(shape) == 3:
        x = synth.field(shape, 7)
    else:
        x = np.stack([synth.field(shape[:3], 70 + f) for f in range(shape[3])], axis=-1)
    t_o = oracle.sthosvd(x, eps)
    t_g = _run(x, eps, torch.float32, precision=precision)
    ok, how, t_f = rank_parity(x, t_g, t_o, 0.1, eps)
    err = gpu_rel_error(x, t_g)
    log("  ranks gpu", t_g.ranks, "oracle", t_o.ranks, how, "err %.4e" % err, "paths", t_g.eig_path)
    assert ok, how
    assert err <= 1.02 * eps
    assert abs(t_g.norm2 - t_o.norm2) <= 1e-5 * t_o.norm2
    # against the oracle run that kept the same ranks
    diff = recon_rel_diff(x, t_g, t_f)
    log("  |X~_gpu - X~_oracle| / |X| = %.3e" % diff)
    assert diff <= 0.2 * eps
    # the sign rule on both sides: each kept column whose eigenvalue is well
    # separated (gaps above 1e-3 of the largest) points the oracle's way (a
    # flipped sign gives -1, a swapped column about 0)
    for k in range(len(shape)):
        lam = np.asarray(t_f.eigvals[k], dtype=np.float64)
        ug, uf = np64(t_g.factors[k]), t_f.factors[k]
        dots = []
        for j in range(t_g.ranks[k]):
            gap = min(lam[j - 1] - lam[j] if j > 0 else np.inf, lam[j] - lam[j + 1] if j + 1 < len(lam) else np.inf)
            if gap > 1e-3 * lam[0]:
                dots.append(float(ug[:, j] @ uf[:, j]))
        log("  mode", k, "separated columns", len(dots), "min dot %.6f" % (min(dots) if dots else 1.0))
        assert all(v >= 0.9 for v in dots), (k, dots)


def test_f64_known_rank_padded_jacobi():
    """Modes of 33, 47 and 64 in FP64 go to the 64 x 64 slot-order Jacobi (the
    first two zero-padded to 64): the oracle's ranks, tails to 1e-12 of the
    squared norm and the kept subspaces to 1e-10 in projector norm."""
    x, _, _ = synth.known_rank_tucker((33, 47, 64), (5, 7, 9), seed=33, rel_noise=1e-3)
    t_o = oracle.sthosvd(x, 1e-2, order=[0, 1, 2])
    t_g = _run(x, 1e-2, torch.float64, order=[0, 1, 2])
    log("padded Jacobi: ranks", t_g.ranks, "sweeps", t_g.eig_sweeps)
    assert t_g.ranks == t_o.ranks == [5, 7, 9]
    assert t_g.eig_path == [1, 1, 1]
    for k in range(3):
        assert abs(t_g.tails[k] - t_o.tails[k]) <= 1e-12 * t_o.norm2
        assert projector_gap(np64(t_g.factors[k]), t_o.factors[k]) < 1e-10


def test_dense_and_subspace_paths_agree():
    x = synth.field((90, 80, 70), 11)
    t_o = oracle.sthosvd(x, 1e-3)
    t_s = _run(x, 1e-3, torch.float32, eig_path=2)
    t_d = _run(x, 1e-3, torch.float32, eig_path=1)
    assert t_s.eig_path[0] == 2 and t_d.eig_path[0] == 1
    for name, t in (("subspace", t_s), ("dense", t_d)):
        log(name, t.ranks, "tails/b", [t.tails[k] / t.budgets[k] for k in range(3)], "sweeps", t.eig_sweeps,
            "norm2", t.norm2)
    log("oracle", t_o.ranks, "tails/b", [t_o.tails[k] / t_o.budgets[k] for k in range(3)], "norm2", t_o.norm2)
    # same Gram matrix, two eigensolvers: unbiased tails on both sides
    assert t_s.ranks == t_d.ranks
    for k in range(3):
        assert abs(t_s.tails[k] - t_d.tails[k]) <= 0.02 * t_d.budgets[k]
    ok, how, _ = rank_parity(x, t_s, t_o, 0.1, 1e-3)
    assert ok, how
    # two power steps leave ~(lambda_noise / lambda_r)^2 of the subspace unresolved
    gaps = [projector_gap(np64(t_s.factors[k]), np64(t_d.factors[k])) for k in range(3)]
    log("projector gaps subspace vs dense", ["%.2e" % g for g in gaps])
    for k in range(3):
        assert gaps[k] < 2e-3
    assert recon_rel_diff(x, t_s, t_o) <= 0.1 * 1e-3


def test_zero_and_nonfinite_inputs():
    z = np.zeros((8, 9, 10))
    t = _run(z, 1e-3, torch.float64)
    assert t.ranks == [1, 1, 1] and t.sse_pred == 0.0
    bad = np.ones((8, 9, 10), dtype=np.float32)
    bad[3, 4, 5] = np.inf
    with pytest.raises(atc.AtcError) as e:
        _run(bad, 1e-3, torch.float32)
    assert e.value.status == -6


def test_deterministic_bits():
    x = synth.field((64, 48, 56), 2)
    a = _run(x, 1e-3, torch.float32, precision="bf16x3")
    b = _run(x, 1e-3, torch.float32, precision="bf16x3")
    assert a.ranks == b.ranks
    assert torch.equal(a.core, b.core)
    for fa, fb in zip(a.factors, b.factors):
        assert torch.equal(fa, fb)


@pytest.mark.parametrize("precision", ["native", "bf16x3"])
def test_tall_short_last_mode(precision):
    """A 13-long last mode over 589,824 rows (several LDS chunks per workgroup,
    rows of 13 floats): the first processed Gram matrix comes from FP64 MFMA
    with exact products, so |A|^2 and that mode's discarded energy match an
    FP64 Gram matrix formed here to rounding, and the rank to the letter."""
    x = synth.field((4096, 144, 13), 13)
    eps = 1e-3
    t = _run(x, eps, torch.float32, precision=precision)
    rows = x.reshape(-1, 13).astype(np.float64)
    g = rows.T @ rows
    norm2 = float(np.trace(g))
    assert abs(t.norm2 - norm2) <= 1e-12 * norm2
    lam = np.sort(np.linalg.eigvalsh(g))[::-1]
    tails = np.concatenate([np.cumsum(lam[::-1])[::-1], [0.0]])  # tails[r] = sum_{j >= r} lam_j
    budget = eps * eps * norm2 / 3
    r = int(np.nonzero(tails[1:] <= budget)[0][0]) + 1
    assert t.order[0] == 2
    assert t.ranks[2] == r, (t.ranks, r)
    assert abs(t.tails[2] - tails[r]) <= 1e-9 * norm2
    err = gpu_rel_error(x, t)
    log("  tall last mode: ranks", t.ranks, "err %.4e" % err)
    assert err <= 1.02 * eps


@pytest.mark.parametrize("precision", ["native", "bf16x3"])
def test_subspace_64_path(precision):
    """Ranks above the m = 32 subspace's reach (24) on modes of 64 < n <= 512:
    the m = 64 path (two orthonormalised 32-column halves, 64 x 64 Rayleigh-Ritz)
    must give the oracle's ranks to the letter on a known-rank tensor."""
    x, _, _ = synth.known_rank_tucker((150, 120, 100), (40, 36, 30), seed=64, rel_noise=1e-4)
    x = x.astype(np.float32)
    eps = 1e-2
    t_o = oracle.sthosvd(x.astype(np.float64), eps)
    t_g = _run(x, eps, torch.float32, precision=precision)
    err = gpu_rel_error(x, t_g)
    log("  m = 64 path: ranks gpu", t_g.ranks, "oracle", t_o.ranks, "paths", t_g.eig_path, "err %.4e" % err)
    assert t_o.ranks == [40, 36, 30]
    assert t_g.ranks == t_o.ranks
    assert t_g.eig_path == [2, 2, 2]
    assert err <= 1.02 * eps
    assert recon_rel_diff(x, t_g, t_o) <= 0.1 * eps


@pytest.mark.parametrize("shape", [(90, 80, 70), (512, 20, 24), (300, 65, 33)])
def test_subspace_one_launch_and_kernel_chain_agree(shape, monkeypatch):
    """The m = 32 subspace path as one cooperative launch (default) and as a
    chain of kernels (ATC_SUB32_KERNELS=1) run the same iteration from the same
    start block: same ranks, tails and kept subspaces up to rounding order.
    Workgroups of 32 rows: 16 of them for n = 512, a last one of 26, 12 and 1
    rows for n = 90, 300 and 65."""
    x = synth.field(shape, 5)
    # both runs project every mode by U^T in one step (no split solver)
    monkeypatch.setenv("ATC_NO_OVERLAP", "1")
    monkeypatch.delenv("ATC_SUB32_KERNELS", raising=False)
    t_c = _run(x, 1e-3, torch.float32, eig_path=2)
    monkeypatch.setenv("ATC_SUB32_KERNELS", "1")
    t_k = _run(x, 1e-3, torch.float32, eig_path=2)
    monkeypatch.delenv("ATC_SUB32_KERNELS")
    log("one launch", t_c.ranks, t_c.eig_path, "kernels", t_k.ranks, t_k.eig_path)
    sub = [k for k, n in enumerate(shape) if 64 < n <= 512]  # n <= 64 goes to the dense solver
    assert sub, shape
    for k in sub:
        assert t_c.eig_path[k] == 2 and t_k.eig_path[k] == 2, (t_c.eig_path, t_k.eig_path)
    assert t_c.ranks == t_k.ranks
    for k in range(len(shape)):
        assert abs(t_c.tails[k] - t_k.tails[k]) <= 1e-9 * t_c.norm2
        gap = projector_gap(np64(t_c.factors[k]), np64(t_k.factors[k]))
        log("  mode", k, "projector gap %.2e" % gap)
        assert gap < 1e-7
        # the sign rule picks the same rows: columns agree to rounding
        assert np.max(np.abs(np64(t_c.factors[k]) - np64(t_k.factors[k]))) < 1e-6
    xc = oracle.reconstruct(np64(t_c.core), [np64(f) for f in t_c.factors])
    xk = oracle.reconstruct(np64(t_k.core), [np64(f) for f in t_k.factors])
    assert np.sqrt(oracle.norm2(xc - xk) / oracle.norm2(x)) < 1e-6
    ok, how, _ = rank_parity(x, t_c, oracle.sthosvd(x, 1e-3), 0.1, 1e-3)
    assert ok, how


@pytest.mark.parametrize("shape,ranks", [((150, 120, 100), (40, 36, 30)), ((500, 70, 90), (50, 40, 44))])
def test_subspace_64_one_launch_and_kernel_chain_agree(shape, ranks, monkeypatch):
    """The m = 64 path's power steps and Rayleigh-Ritz matrix as one cooperative
    launch (default) and as a chain of kernels (ATC_SUB32_KERNELS=1): the same
    ranks, tails and kept subspaces up to rounding order, and the oracle's
    ranks.  Workgroups of 32 rows: 16 for n = 500 (the last one of 20 rows),
    3 for n = 70 (the last of 6)."""
    x, _, _ = synth.known_rank_tucker(shape, ranks, seed=65, rel_noise=1e-4)
    x = x.astype(np.float32)
    eps = 1e-2
    monkeypatch.delenv("ATC_SUB32_KERNELS", raising=False)
    t_c = _run(x, eps, torch.float32)
    monkeypatch.setenv("ATC_SUB32_KERNELS", "1")
    t_k = _run(x, eps, torch.float32)
    monkeypatch.delenv("ATC_SUB32_KERNELS")
    log("m = 64 one launch", t_c.ranks, t_c.eig_path, "kernels", t_k.ranks, t_k.eig_path)
    assert t_c.eig_path == [2, 2, 2] and t_k.eig_path == [2, 2, 2]
    assert t_c.ranks == t_k.ranks == list(ranks)
    for k in range(len(shape)):
        assert abs(t_c.tails[k] - t_k.tails[k]) <= 1e-9 * t_c.norm2
        gap = projector_gap(np64(t_c.factors[k]), np64(t_k.factors[k]))
        log("  mode", k, "projector gap %.2e" % gap)
        assert gap < 1e-7
        assert np.max(np.abs(np64(t_c.factors[k]) - np64(t_k.factors[k]))) < 1e-6
    assert t_c.ranks == oracle.sthosvd(x.astype(np.float64), eps).ranks


def test_grid_barrier_wait_gives_up_without_hanging(monkeypatch):
    """The one-launch eigensolver's barrier waits are bounded: a limit of zero
    polls (forced from the host) makes every wait give up at once, every
    workgroup still runs to its end, the call reports an internal error instead
    of hanging, and the next call (normal limit) gives the same bits as before."""
    x = synth.field((160, 96, 80), 7)
    ref = _run(x, 1e-3, torch.float32, eig_path=2)
    monkeypatch.setenv("ATC_GRID_SPIN_LIMIT", "0")
    with pytest.raises(atc.AtcError) as e:
        _run(x, 1e-3, torch.float32, eig_path=2)
    assert e.value.status == -7, e.value.status
    monkeypatch.delenv("ATC_GRID_SPIN_LIMIT")
    torch.cuda.synchronize()
    again = _run(x, 1e-3, torch.float32, eig_path=2)
    assert again.ranks == ref.ranks
    assert torch.equal(again.core, ref.core)
    for fa, fb in zip(again.factors, ref.factors):
        assert torch.equal(fa, fb)


@pytest.mark.parametrize("precision", ["native", "bf16x3"])
@pytest.mark.parametrize("shape,min_bytes", [((90, 80, 70), "0"), ((160, 130, 100), "0"), ((256, 256, 256), None)])
def test_split_solver_matches_one_launch(shape, min_bytes, precision, monkeypatch):
    """The m = 32 solver split in two launches, the mode product by the basis
    Q^T running beside the Rayleigh-Ritz step and then rotated by W_r^T
    (every mode but the last), against the one-launch solver that projects by
    U^T = (Q W_r)^T in one step.  The two-step projection rounds differently
    (two float32 mode products of 32 and n terms instead of one), so later
    Gram matrices differ at float32 rounding, |dG| <= 64 u |G| (u = 2^-24):
    ranks equal, tails within 1e-6 |A|^2, kept subspaces within the
    Davis-Kahan bound |dG| / (lam_r - lam_{r+1}) at the cut (eigenvalues from
    the oracle), reconstructions within 1e-5 of |A|.  The split form is taken for
    tensors of 64 MiB and more (the 256^3 field's first mode); the smaller
    shapes lower that threshold to reach it on every mode but the last."""
    x = synth.field(shape, 5)
    if min_bytes is not None:
        monkeypatch.setenv("ATC_SPLIT_MIN_BYTES", min_bytes)
    monkeypatch.setenv("ATC_NO_OVERLAP", "1")
    t_1 = _run(x, 1e-3, torch.float32, precision=precision, eig_path=2)
    monkeypatch.delenv("ATC_NO_OVERLAP")
    t_s = _run(x, 1e-3, torch.float32, precision=precision, eig_path=2)
    t_o = oracle.sthosvd(x, 1e-3)
    assert t_1.ranks == t_s.ranks
    for k in range(len(shape)):
        assert t_1.eig_path[k] == t_s.eig_path[k]
        assert abs(t_1.tails[k] - t_s.tails[k]) <= 1e-6 * t_1.norm2
        lam, r = np.asarray(t_o.eigvals[k]), t_1.ranks[k]
        cut = lam[r - 1] - (lam[r] if r < lam.size else 0.0)
        bound = 64 * 2.0 ** -24 * lam[0] / cut
        gap = projector_gap(np64(t_1.factors[k]), np64(t_s.factors[k]))
        log("split vs one launch %s %s mode %d: projector gap %.2e (bound %.2e)" % (shape, precision, k, gap, bound))
        assert gap <= bound
    x1 = oracle.reconstruct(np64(t_1.core), [np64(f) for f in t_1.factors])
    xs = oracle.reconstruct(np64(t_s.core), [np64(f) for f in t_s.factors])
    assert np.sqrt(oracle.norm2(x1 - xs) / oracle.norm2(x)) < 1e-5
    ok, how, _ = rank_parity(x, t_s, t_o, 0.1, 1e-3)
    assert ok, how
