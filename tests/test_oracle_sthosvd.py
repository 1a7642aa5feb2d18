"""Pins for the oracle's ST-HOSVD (Algorithm 1 with the Section 4.1 choices).

Closed forms (super-diagonal tensor), the matrix case (d = 2 is the truncated SVD,
checked against numpy.linalg.svd, Eckart-Young), exact recovery of tensors of
known multilinear rank, the identity |X - X~|^2 = sum of the discarded eigenvalues
(Section 4.1.3), orthonormal factors (Section 3.2), all-orthogonality of the core
in the last processed mode, invariances, and the published-shape configurations.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import load_golden


def superdiag_tensor(shape, diag):
    x = np.zeros(shape)
    for i, s in enumerate(diag):
        x[i, i, i] = s
    return x


@pytest.mark.parametrize("case", load_golden("superdiag.json")["cases"])
def test_superdiagonal_closed_form(case):
    g = load_golden("superdiag.json")
    x = superdiag_tensor(g["shape"], g["diag"])
    nrm2 = float(np.sum(np.square(g["diag"])))
    eps = float(np.sqrt(case["budget"] / nrm2))
    t = oracle.sthosvd(x, eps, rule=case["rule"])
    assert t.order == [0, 1, 2]
    assert t.ranks == case["ranks"]
    assert np.allclose(t.tails, case["tails"], atol=1e-12)
    assert abs(t.sse_pred - case["sse"]) <= 1e-12
    assert abs(oracle.norm2(x - oracle.reconstruct(t.core, t.factors)) - case["sse"]) <= 1e-12


@pytest.mark.parametrize("m,n", [(7, 5), (12, 30), (40, 40)])
@pytest.mark.parametrize("eps", [0.05, 0.3, 0.8])
def test_matrix_case_is_truncated_svd(m, n, eps):
    rng = np.random.default_rng(m * 100 + n)
    a = rng.standard_normal((m, n)) * np.logspace(0, -2, n)
    s = np.linalg.svd(a, compute_uv=False)
    u_ref, _, vt_ref = np.linalg.svd(a)
    t = oracle.sthosvd(a, eps, rule="equal")
    budget = eps ** 2 * np.sum(s ** 2) / 2
    # mode order by increasing length; the smaller mode is truncated by Eckart-Young
    tails = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1][1:], [0.0]])
    k0 = t.order[0]
    r_ref = 1 + int(np.argmax(tails <= budget))
    assert t.ranks[k0] == r_ref
    assert abs(t.tails[k0] - tails[r_ref - 1]) <= 1e-10 * np.sum(s ** 2)
    # the kept subspace of the first processed mode matches the SVD's
    ref_basis = u_ref[:, :r_ref] if k0 == 0 else vt_ref[:r_ref].T
    p = t.factors[k0] @ t.factors[k0].T
    if r_ref < min(m, n) and s[r_ref - 1] > s[r_ref] * (1 + 1e-6):
        assert np.abs(p - ref_basis @ ref_basis.T).max() < 1e-8
    assert oracle.rel_error(a, t.core, t.factors) <= eps * (1 + 1e-12)


@pytest.mark.parametrize("dims,ranks", [((10, 12, 14), (3, 5, 2)), ((8, 9, 7, 6), (2, 3, 4, 1)), ((20, 6, 30), (4, 6, 5))])
def test_exact_recovery_of_known_multilinear_rank(dims, ranks):
    # eps must exceed the FP64 rounding floor of the zero eigenvalues (~1e-16 |G|
    # each, so eps > ~1e-7) and stay below the smallest signal share (>= 7e-5 here)
    x, core, facs = synth.known_rank_tucker(dims, ranks, seed=7)
    for eps in (1e-6, 1e-4, 3e-3):
        t = oracle.sthosvd(x, eps)
        assert t.ranks == list(ranks)
        err = oracle.rel_error(x, t.core, t.factors)
        assert err < 1e-13
        for k in range(len(dims)):
            p = t.factors[k] @ t.factors[k].T
            pr = facs[k] @ facs[k].T
            assert np.abs(p - pr).max() < 1e-12


def test_zero_tensor_gives_rank_one():
    t = oracle.sthosvd(np.zeros((4, 3, 5)), 1e-3)
    assert t.ranks == [1, 1, 1] and t.sse_pred == 0.0 and t.norm2 == 0.0


@pytest.fixture(scope="module")
def small_field():
    return synth.field((24, 20, 28), 5).astype(np.float64)


@pytest.mark.parametrize("rule", ["adaptive", "equal"])
@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-3, 1e-4])
def test_sse_identity_error_bound_and_orthonormality(small_field, rule, eps):
    x = small_field
    t = oracle.sthosvd(x, eps, rule=rule)
    sse = oracle.norm2(x - oracle.reconstruct(t.core, t.factors))
    nrm2 = oracle.norm2(x)
    # Section 4.1.3: truncation SSE equals the discarded squared singular values
    assert abs(sse - t.sse_pred) <= 1e-10 * nrm2
    # orthonormal factors -> |core|^2 = |X|^2 - SSE
    assert abs(oracle.norm2(t.core) - (nrm2 - t.sse_pred)) <= 1e-10 * nrm2
    assert np.sqrt(sse / nrm2) <= eps * (1 + 1e-9)
    assert t.sse_pred <= eps ** 2 * nrm2 * (1 + 1e-12)
    for u in t.factors:
        assert np.abs(u.T @ u - np.eye(u.shape[1])).max() < 1e-13
    # all-orthogonality in the last processed mode: its Gram matrix of the core
    # is the diagonal of the kept eigenvalues of that step
    k = t.order[-1]
    gk = oracle.gram(t.core, k)
    kept = t.eigvals[k][: t.ranks[k]]
    assert np.abs(gk - np.diag(kept)).max() <= 1e-10 * nrm2
    # sign rule: every column's largest-magnitude entry is positive
    for u in t.factors:
        idx = np.argmax(np.abs(u), axis=0)
        assert np.all(u[idx, np.arange(u.shape[1])] > 0)


def test_processing_order_default_and_user():
    assert oracle.processing_order([200, 500, 500, 13]) == [3, 0, 1, 2]
    assert oracle.processing_order([64, 64, 64]) == [0, 1, 2]
    assert oracle.processing_order([5, 3, 5, 3]) == [1, 3, 0, 2]
    assert oracle.processing_order([5, 3, 4], [2, 0, 1]) == [2, 0, 1]
    with pytest.raises(ValueError):
        oracle.processing_order([5, 3, 4], [0, 0, 1])


def test_invariances(small_field):
    x = small_field
    eps = 1e-3
    t = oracle.sthosvd(x, eps)
    # scaling: same ranks, core scales, factors unchanged
    ts = oracle.sthosvd(3.5 * x, eps)
    assert ts.ranks == t.ranks
    assert np.allclose(ts.core, 3.5 * t.core, rtol=1e-9, atol=1e-9 * np.abs(t.core).max())
    # orthogonal change of basis on mode 1 rotates U_1 and leaves the rest
    q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((x.shape[1],) * 2))
    tq = oracle.sthosvd(oracle.mode_product(x, 1, q), eps)
    assert tq.ranks == t.ranks
    p = tq.factors[1] @ tq.factors[1].T
    pr = (q @ t.factors[1]) @ (q @ t.factors[1]).T
    assert np.abs(p - pr).max() < 1e-8
    # relabelling the modes together with the order permutes every output
    perm = [2, 0, 1]
    xp = np.transpose(x, perm)
    order_p = [perm.index(k) for k in t.order]
    tp = oracle.sthosvd(xp, eps, order=order_p)
    assert [tp.ranks[perm.index(k)] for k in range(3)] == t.ranks
    assert np.allclose(np.transpose(t.core, perm), tp.core, rtol=1e-8, atol=1e-8 * np.abs(t.core).max())


def test_fixed_ranks_override(small_field):
    t = oracle.sthosvd(small_field, 1e-2, fixed_ranks=[3, 4, 5])
    assert t.ranks == [3, 4, 5] and t.core.shape == (3, 4, 5)
    assert abs(oracle.norm2(small_field - oracle.reconstruct(t.core, t.factors)) - t.sse_pred) <= 1e-10 * t.norm2


def test_config_64cube_known_rank_plus_noise():
    """64^3 float64 Tucker(core 8^3) + noise at 1e-3 relative, eps = 1e-2: ranks (8,8,8)."""
    x = synth.tucker_c1("relative")
    t = oracle.sthosvd(x, 1e-2, order=[0, 1, 2])
    assert t.ranks == [8, 8, 8]
    err = oracle.rel_error(x, t.core, t.factors)
    assert 5e-4 < err < 2e-3
    assert t.converged
    # with the noise read as an absolute std of 1e-3 (2.2% relative) the budget
    # cannot absorb it and the ranks jump far past 8
    ta = oracle.sthosvd(synth.tucker_c1("absolute"), 1e-2, order=[0, 1, 2])
    assert min(ta.ranks) > 40
    tn = oracle.sthosvd(synth.tucker_c1("none"), 1e-2)
    assert tn.ranks == [8, 8, 8] and oracle.rel_error(synth.tucker_c1("none"), tn.core, tn.factors) < 1e-13


@pytest.mark.slow
def test_field256_regression_ranks():
    """256^3 field (seed 0): the ranks and errors computed independently with a
    LAPACK-eigh FP64 ST-HOSVD of the same generator when the workloads were specified."""
    x = synth.field((256,) * 3, 0)
    expect = {1e-2: ([14, 11, 12], 9.55e-3), 1e-3: ([18, 15, 18], 8.27e-4), 1e-4: ([22, 18, 20], 6.85e-5)}
    for eps, (ranks, err) in expect.items():
        t = oracle.sthosvd(x, eps)
        assert t.ranks == ranks
        assert abs(np.sqrt(t.sse_pred / t.norm2) - err) <= 0.006 * err
