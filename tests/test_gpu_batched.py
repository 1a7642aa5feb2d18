"""GPU parity of the batched persistent ST-HOSVD (atc_sthosvd_batched) against the
FP64 oracle run block by block, plus HIP-graph replay and the autotuner.

Bars per block (bf16x3 and FP32 products, FP64 eigensolver): ranks equal or
boundary-degenerate (oracle discarded energy at the GPU rank within 10% of the
mode budget, 20% for the plain FP32 path), achieved error <= 1.02 eps (1.05 eps for the plain FP32 path), |X~_gpu - X~_oracle| / |X| <= 0.2 eps
when ranks agree, and |A|^2 to 1e-5.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2107_01384_amd as atc
import synth
from gpu_helpers import log

pytestmark = pytest.mark.gpu


def _arena(dims, seed0):
    arena, _ = synth.batch_arena(dims, seed0)
    return torch.from_numpy(arena).cuda()


def _check_block(plan, arena_np, core, fac, recs, b, eps, err_factor=1.02, band=0.1):
    d = [int(v) for v in plan.dims[b]]
    x = arena_np[plan.input_off[b]: plan.input_off[b] + np.prod(d)].reshape(d)
    rec = recs[b]
    ranks = [int(r) for r in rec["ranks"]]
    assert rec["status"] == 0, (b, rec["status"])
    t_o = oracle.sthosvd(x, eps)
    g_core = plan.core_of(core, b, ranks).double().cpu().numpy()
    g_facs = [plan.factor_of(fac, b, k, ranks[k]).double().cpu().numpy() for k in range(3)]
    err = oracle.rel_error(x, g_core, g_facs)
    assert err <= err_factor * eps, (b, d, ranks, err)
    assert abs(rec["norm2"] - t_o.norm2) <= 1e-5 * t_o.norm2
    if ranks == t_o.ranks:
        xg = oracle.reconstruct(g_core, g_facs)
        xo = oracle.reconstruct(t_o.core, t_o.factors)
        diff = np.sqrt(oracle.norm2(xg - xo) / t_o.norm2)
        assert diff <= 0.2 * eps, (b, d, diff)
        return True
    for k in range(3):
        if ranks[k] != t_o.ranks[k]:
            tails = oracle.tail_sums(t_o.eigvals[k])
            bud = t_o.budgets[k]
            near = min(abs(tails[ranks[k]] - bud), abs(tails[t_o.ranks[k]] - bud))
            assert near <= band * bud, (b, d, ranks, t_o.ranks)
    return False


@pytest.mark.parametrize("precision", ["bf16x3", "native"])
def test_batched_small_mixed_sizes(precision):
    rng = np.random.default_rng(5)
    # standard block sizes plus odd ones that exercise every loader layout
    sizes = np.array([16, 24, 32, 48, 64, 1, 5, 13, 17, 33], dtype=np.int32)
    dims = rng.choice(sizes, size=(48, 3)).astype(np.int32)
    dims[0] = (64, 64, 64)
    dims[1] = (1, 1, 1)
    dims[2] = (64, 2, 3)
    arena_np, _ = synth.batch_arena(dims, 500)
    arena = torch.from_numpy(arena_np).cuda()
    eps = 1e-3
    plan = atc.BatchPlan(dims, eps, precision)
    core, fac, res, ws = plan.allocate()
    plan.run(arena, core, fac, res, ws)
    torch.cuda.synchronize()
    recs = plan.results(res)
    # the plain FP32 Gram is at its precision floor at 1e-3: its unbiased tail
    # estimates scatter by a few percent of the budget (bf16x3 keeps 1.02)
    # and its rank can sit on the other side of a boundary the oracle places
    # within 20% of the budget (bf16x3: 10%)
    factor, band = (1.02, 0.1) if precision == "bf16x3" else (1.05, 0.2)
    exact = sum(_check_block(plan, arena_np, core, fac, recs, b, eps, factor, band) for b in range(len(dims)))
    log("batched", precision, "blocks", len(dims), "exact-rank blocks", exact)
    assert exact >= len(dims) - (2 if precision == "bf16x3" else 4)


def test_batched_graph_replay_and_autotune(tmp_path):
    dims = synth.batch_dims(96, seed=7)
    arena_np, _ = synth.batch_arena(dims, 900)
    arena = torch.from_numpy(arena_np).cuda()
    plan = atc.BatchPlan(dims, 1e-3, "bf16x3")
    core, fac, res, ws = plan.allocate()
    cache = str(tmp_path / "tune.jsonl")
    choice = plan.autotune(arena, core, fac, res, ws, reps=2, cache_path=cache)
    assert 0 <= choice < 4
    assert os.path.exists(cache) and open(cache).read().count("\n") == 1
    plan2 = atc.BatchPlan(dims, 1e-3, "bf16x3")
    assert plan2.autotune(arena, core, fac, res, ws, reps=2, cache_path=cache) == choice  # read from cache
    assert open(cache).read().count("\n") == 1
    # eager reference; the arenas are cleared first, as before every replay,
    # since slot entries beyond a block's core and factors are never written
    core.zero_()
    fac.zero_()
    res.zero_()
    plan.run(arena, core, fac, res, ws)
    torch.cuda.synchronize()
    ref_core, ref_fac, ref_res = core.clone(), fac.clone(), res.clone()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.capture(arena, core, fac, res, ws, stream=stream)
    for rep in range(3):
        core.zero_()
        fac.zero_()
        res.zero_()
        torch.cuda.synchronize()
        plan.replay(stream=stream)
        stream.synchronize()
        _ = (arena * 2.0).sum().item()  # unrelated eager work between replays
        assert torch.equal(res, ref_res), rep
        assert torch.equal(core, ref_core), rep
        assert torch.equal(fac, ref_fac), rep
    log("graph replays identical; autotune choice", choice)


def test_batched_full_size_sampled():
    """4096 blocks (sizes from {16,24,32,48,64}^3), one launch; 40 sampled blocks vs the oracle."""
    dims = synth.batch_dims(4096, seed=2024)
    arena_np, _ = synth.batch_arena(dims, 10_000)
    arena = torch.from_numpy(arena_np).cuda()
    eps = 1e-3
    plan = atc.BatchPlan(dims, eps, "bf16x3")
    core, fac, res, ws = plan.allocate()
    plan.run(arena, core, fac, res, ws)
    torch.cuda.synchronize()
    recs = plan.results(res)
    assert np.all(recs["status"] == 0)
    assert np.all(recs["ranks"] >= 1) and np.all(recs["ranks"] <= plan.dims)
    # the identity |X - X~|^2 = sum of discarded eigenvalues holds within budget for every block
    assert np.all(recs["sse_pred"] <= (eps ** 2) * recs["norm2"] * (1 + 1e-9))
    sample = np.random.default_rng(1).choice(4096, size=40, replace=False)
    exact = sum(_check_block(plan, arena_np, core, fac, recs, int(b), eps) for b in sample)
    log("full batch sampled exact-rank blocks", exact, "of", len(sample))
    assert exact >= len(sample) - 3
