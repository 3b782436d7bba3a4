"""GPU parity of the batched solver (gep_solve_batched): the 256-instance batch
with orders drawn log-uniformly in [64, 2048] (instance seeds 4000+i), checked
per instance by invariants, against the oracle on a subset, against single
gep_solve calls, and through HIP-graph capture and replay."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import say, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _gep():
    import paper_1504_06443_amd as gep
    return gep


def _invariants(A, B, lam, Y):
    import torch
    n1 = A.abs().sum(0).max()
    AY = A @ Y
    BY = B @ Y
    res = ((AY - BY * lam[None, :]).abs().sum(0).max() / (n1 * Y.abs().sum(0).max())).item()
    G = Y.t() @ BY
    G.diagonal().sub_(1.0)
    return res, G.abs().max().item()


def test_batch_256_workload(gpu):
    import torch
    gep = _gep()
    sizes = synth.batch_sizes()
    say(f"[batched] generating 256 instances, sum M^2 = {sum(m * m for m in sizes):.3e}")
    As, Bs = [], []
    for i, M in enumerate(sizes):
        A, B = synth.batch_instance(i, M)
        As.append(to_gpu(A))
        Bs.append(to_gpu(B))
    say("[batched] solving")
    bs = gep.BatchedSolver(sizes)
    bs.load(As, Bs)
    bs.run()
    torch.cuda.synchronize()
    assert int(bs.info.abs().sum().item()) == 0
    out = bs.results()
    worst_res = worst_orth = 0.0
    bad = []
    for i, (lam, Y) in enumerate(out):
        assert bool((lam[1:] >= lam[:-1]).all())
        res, orth = _invariants(As[i], Bs[i], lam, Y.contiguous())
        worst_res = max(worst_res, res)
        worst_orth = max(worst_orth, orth)
        if res > 1e-12 or orth > 1e-12:
            bad.append((i, sizes[i], res, orth))
    say(f"[batched] worst residual {worst_res:.2e}, worst orthogonality {worst_orth:.2e}")
    assert not bad, f"instances (index, M, residual, orthogonality) failing: {bad[:16]}"
    # oracle on the smaller instances
    small = sorted(range(len(sizes)), key=lambda i: sizes[i])[:6]
    for i in small:
        A, B = synth.batch_instance(i, sizes[i])
        r = oracle.solve(A, B)
        err = np.abs(to_np(out[i][0]) - r.lam).max() / r.norm1
        assert err <= 1e-11, (i, sizes[i], err)
    # identical to the single-problem path
    for i in (small[0], int(np.argmax(sizes))):
        lam1, Y1 = gep.solve(As[i], Bs[i])
        assert torch.equal(lam1, out[i][0]) and torch.equal(Y1, out[i][1])


def test_batch_graph_replay(gpu):
    """Capture one batched call in a graph, replay it several times with eager
    work and synchronisations in between; every replay must equal the eager run."""
    import torch
    gep = _gep()
    sizes = [64, 65, 100, 129, 257, 300, 511, 700, 1024, 77, 64, 333]
    As, Bs = [], []
    for i, M in enumerate(sizes):
        A, B = synth.batch_instance(100 + i, M)
        As.append(to_gpu(A))
        Bs.append(to_gpu(B))
    bs = gep.BatchedSolver(sizes)
    bs.load(As, Bs)
    bs.run()
    torch.cuda.synchronize()
    ref = [(l.clone(), Y.clone()) for l, Y in bs.results()]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        bs.run()  # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            bs.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for l, Y in bs.results():
            l.zero_()
            Y.zero_()
        _ = torch.randn(1000, 1000, device="cuda").sum().item()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        for (l, Y), (l0, Y0) in zip(bs.results(), ref):
            assert torch.equal(l, l0) and torch.equal(Y, Y0), rep


def test_batched_graph_per_stream_replay(gpu):
    """BatchedGraph: the batch split into groups, one captured graph per group and
    stream, replayed concurrently; every replay (with eager work and
    synchronisations in between) must equal one eager call of the whole batch,
    and the instance order of results() must be the caller's."""
    import torch
    gep = _gep()
    sizes = [64, 65, 100, 129, 257, 300, 511, 700, 1024, 77, 64, 333, 2048, 190]
    As, Bs = [], []
    for i, M in enumerate(sizes):
        A, B = synth.batch_instance(200 + i, M)
        As.append(to_gpu(A))
        Bs.append(to_gpu(B))
    bs = gep.BatchedSolver(sizes)
    bs.load(As, Bs)
    bs.run()
    torch.cuda.synchronize()
    ref = [(l.clone(), Y.clone()) for l, Y in bs.results()]
    bg = gep.BatchedGraph(sizes, groups=5)
    assert sorted(i for m in bg.members for i in m) == list(range(len(sizes)))
    bg.load(As, Bs)
    bg.capture()
    for rep in range(3):
        for l, Y in bg.results():
            l.zero_()
            Y.zero_()
        _ = torch.randn(1000, 1000, device="cuda").sum().item()  # eager work between replays
        bg.replay()
        torch.cuda.synchronize()
        assert int(bg.info.abs().sum().item()) == 0
        for (l, Y), (l0, Y0) in zip(bg.results(), ref):
            assert torch.equal(l, l0) and torch.equal(Y, Y0), rep
