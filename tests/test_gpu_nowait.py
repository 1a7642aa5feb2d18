"""The fixed-rank ST-HOSVD call that never waits on the host (opts.no_host_wait)
and its capture in a graph, through the C ABI.

Bars:
  * eager no-host-wait call (subspace solvers in their one-launch form) vs
    the ordinary call with the same fixed ranks (kernel chains, no split
    solver): same ranks, tails and |A|^2 to 1e-6 relative, kept subspaces
    within 1e-6, reconstructions within 1e-5 of |X| (the two forms agree to
    1e-7 in the kept subspaces on their own);
  * against the FP64 oracle at the same fixed ranks: predicted SSE within
    1e-5 |A|^2 + 1% of the oracle's, reconstruction within 1e-4 of |X|;
  * graph replays on changing inputs (eager library calls and synchronisations
    between them): core, factors and the figures read by atc_sthosvd_finish
    equal bit for bit to the eager no-host-wait call on the same input (its
    subspace solvers as kernel chains, the form a capture records).
Inputs: known multilinear rank plus 1% noise, so every kept Ritz value is a
signal eigenvalue well above rounding.  The ranks cover each eigensolver the
fixed rank picks: r <= 24 (m = 32 subspace), 24 < r <= 56 (m = 64), r > 56
with n > 64 (dense, global memory), n <= 64 (dense in LDS) and r = n.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2107_01384_amd as atc
import synth
from gpu_helpers import log, np64, projector_gap, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ((96, 80, 72), (12, 40, 72), "bf16x3", torch.float32),
    ((60, 100, 50), (60, 70, 20), "native", torch.float32),
    ((40, 30, 20), (5, 6, 7), "native", torch.float64),
]


def _input(shape, ranks, seed):
    x, _, _ = synth.known_rank_tucker(shape, ranks, seed=seed, rel_noise=1e-2)
    return x


def _buffers(shape, dtype, ws_bytes):
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    core = torch.empty(int(np.prod(shape)), dtype=dtype, device="cuda")
    facs = [torch.empty(n * n, dtype=dtype, device="cuda") for n in shape]
    return ws, core, facs


def _snapshot(t):
    return t.core.clone(), [f.clone() for f in t.factors]


@pytest.mark.parametrize("shape,ranks,precision,dtype", CASES)
def test_no_host_wait_matches_ordinary_call_and_oracle(shape, ranks, precision, dtype, monkeypatch):
    _check_against_ordinary_and_oracle(shape, ranks, precision, dtype, monkeypatch)


@pytest.mark.parametrize("precision", ["bf16x3", "native"])
def test_no_host_wait_split_solver(precision, monkeypatch):
    """Mode 0 (n = 96, r = 12) is the second of three in increasing-length
    order: with the size threshold at zero it takes the split m = 32 solver
    (basis, the product by it on the second stream, the rotation queued with
    the device-side rank) with no host wait in between."""
    monkeypatch.setenv("ATC_SPLIT_MIN_BYTES", "0")
    _check_against_ordinary_and_oracle((96, 80, 120), (12, 40, 100), precision, torch.float32, monkeypatch)


def _check_against_ordinary_and_oracle(shape, ranks, precision, dtype, monkeypatch):
    x = _input(shape, ranks, 31)
    xd = to_dev(x, dtype)
    kw = dict(precision=precision, fixed_ranks=list(ranks))
    need = atc.sthosvd_workspace_size(shape, dtype, no_host_wait=True, **kw)
    ws, core, facs = _buffers(shape, dtype, need)
    log("no-host-wait", shape, ranks, precision, dtype)
    t_n = atc.sthosvd(xd, workspace=ws, out=(core, facs), no_host_wait=True, **kw)
    assert t_n.norm2 == 0.0 and t_n.sse_pred == 0.0  # filled by the finish call
    fig = atc.sthosvd_finish(shape, dtype, ws, **kw)
    monkeypatch.setenv("ATC_NO_OVERLAP", "1")
    monkeypatch.setenv("ATC_SUB32_KERNELS", "1")
    t_o = atc.sthosvd(xd, **kw)
    torch.cuda.synchronize()
    log("  ranks", t_n.ranks, "paths", t_n.eig_path, "ordinary paths", t_o.eig_path)
    assert t_n.ranks == t_o.ranks == list(ranks)
    assert t_n.order == t_o.order
    assert abs(fig["norm2"] - t_o.norm2) <= 1e-6 * t_o.norm2
    assert abs(fig["sse_pred"] - t_o.sse_pred) <= 1e-6 * t_o.norm2
    for k in range(len(shape)):
        assert abs(fig["tails"][k] - t_o.tails[k]) <= 1e-6 * t_o.norm2, k
        gap = projector_gap(np64(t_n.factors[k]), np64(t_o.factors[k]))
        log("  mode", k, "projector gap %.2e" % gap)
        assert gap < 1e-6
    xn = oracle.reconstruct(np64(t_n.core), [np64(f) for f in t_n.factors])
    xo = oracle.reconstruct(np64(t_o.core), [np64(f) for f in t_o.factors])
    nx = oracle.norm2(x)
    assert np.sqrt(oracle.norm2(xn - xo) / nx) < 1e-5
    t_r = oracle.sthosvd(x, 1e-3, fixed_ranks=list(ranks))
    assert abs(fig["sse_pred"] - t_r.sse_pred) <= 1e-5 * t_r.norm2 + 1e-2 * t_r.sse_pred
    xr = oracle.reconstruct(t_r.core, t_r.factors)
    assert np.sqrt(oracle.norm2(xn - xr) / nx) < 1e-4


@pytest.mark.parametrize("shape,ranks,precision,dtype", CASES[:2])
def test_no_host_wait_graph_replays(shape, ranks, precision, dtype, monkeypatch):
    # under capture the subspace solvers run as kernel chains: the eager
    # references take the same form
    monkeypatch.setenv("ATC_SUB32_KERNELS", "1")
    kw = dict(precision=precision, fixed_ranks=list(ranks))
    need = atc.sthosvd_workspace_size(shape, dtype, no_host_wait=True, **kw)
    xs = [to_dev(_input(shape, ranks, s), dtype) for s in (41, 42)]
    # eager references, one per input
    ref = []
    for xd in xs:
        ws, core, facs = _buffers(shape, dtype, need)
        t = atc.sthosvd(xd, workspace=ws, out=(core, facs), no_host_wait=True, **kw)
        ref.append((_snapshot(t), atc.sthosvd_finish(shape, dtype, ws, **kw)))
    # capture, with static input, workspace and outputs
    x_static = xs[0].clone()
    ws, core, facs = _buffers(shape, dtype, need)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        atc.sthosvd(x_static, workspace=ws, out=(core, facs), no_host_wait=True, **kw)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        t_g = atc.sthosvd(x_static, workspace=ws, out=(core, facs), no_host_wait=True, **kw)
    assert t_g.ranks == list(ranks)
    other = to_dev(_input(shape, ranks, 7), dtype)
    for rep, j in enumerate((1, 0, 1)):
        x_static.copy_(xs[j])
        torch.cuda.synchronize()
        log("replay", rep, "input", j, shape, ranks, precision)
        graph.replay()
        fig = atc.sthosvd_finish(shape, dtype, ws, **kw)
        (c_ref, f_ref), fig_ref = ref[j]
        assert torch.equal(t_g.core, c_ref), rep
        for k in range(len(shape)):
            assert torch.equal(t_g.factors[k], f_ref[k]), (rep, k)
        assert fig == fig_ref, (rep, fig, fig_ref)
        # the program's own work between replays: an ordinary library call
        # and torch kernels on the same stream
        atc.sthosvd(other, 1e-2, precision=precision)
        torch.cuda.synchronize()


def test_no_host_wait_calls_overlap_on_streams(monkeypatch):
    """One host thread queues two no-host-wait calls on two streams (both taking
    the split m = 32 solver, which shares the thread's second stream) and then
    an ordinary call on a third, with no synchronisation in between: every
    result equals, bit for bit, the same call made alone."""
    monkeypatch.setenv("ATC_SPLIT_MIN_BYTES", "0")
    shape, ranks = (96, 80, 120), (12, 40, 100)
    kw = dict(precision="bf16x3", fixed_ranks=list(ranks))
    need = atc.sthosvd_workspace_size(shape, torch.float32, no_host_wait=True, **kw)
    xs = [to_dev(_input(shape, ranks, s), torch.float32) for s in (51, 52, 53)]
    bufs = [_buffers(shape, torch.float32, need) for _ in range(2)]

    def nowait(j, stream=None):
        ws, core, facs = bufs[j]
        return atc.sthosvd(xs[j], workspace=ws, out=(core, facs), no_host_wait=True, stream=stream, **kw)

    ref = []
    for j in range(2):
        t = nowait(j)
        ref.append((_snapshot(t), atc.sthosvd_finish(shape, torch.float32, bufs[j][0], **kw)))
    t3 = atc.sthosvd(xs[2], 1e-3, precision="bf16x3")
    torch.cuda.synchronize()
    ref3 = _snapshot(t3)
    for j in range(2):
        bufs[j][1].zero_()
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(2)]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    log("overlapping calls", shape, ranks)
    ts = [nowait(j, streams[j]) for j in range(2)]
    o3 = atc.sthosvd(xs[2], 1e-3, precision="bf16x3")
    figs = [atc.sthosvd_finish(shape, torch.float32, bufs[j][0], stream=streams[j], **kw) for j in range(2)]
    torch.cuda.synchronize()
    for j in range(2):
        (c_ref, f_ref), fig_ref = ref[j]
        assert torch.equal(ts[j].core, c_ref), j
        for k in range(3):
            assert torch.equal(ts[j].factors[k], f_ref[k]), (j, k)
        assert figs[j] == fig_ref, j
    assert o3.ranks == t3.ranks
    assert torch.equal(o3.core, ref3[0])
    for k in range(3):
        assert torch.equal(o3.factors[k], ref3[1][k]), k
