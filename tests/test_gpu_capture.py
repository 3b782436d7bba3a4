"""Single solves captured in a HIP graph (torch.cuda.CUDAGraph) and replayed, through
the C ABI: gep_solve (eigenpairs, eigenvalues only, mixed precision),
gep_solve_noalloc and gep_solve_lowest.  Under capture the panel QR and the bulge
chase take their plain-launch forms; the kernels' arithmetic is the same, so
every replay, with eager work and synchronisations in between, must equal the
eager call bitwise, and the eager call must match the oracle."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import say, to_gpu, to_np

pytestmark = pytest.mark.gpu

P = ctypes.c_void_p


def _lib():
    from paper_1504_06443_amd import _binding
    return _binding.lib()


class _Call:
    """Buffers allocated once; enqueue() issues the entry point on the current
    stream (capturable: no allocation, no synchronisation)."""

    def __init__(self, entry, dA, dB, job=1, prec=0, k=None):
        import torch
        L = _lib()
        M = dA.shape[0]
        dev = dA.device
        self.entry, self.M, self.job, self.prec, self.k = entry, M, job, prec, k
        self.dA, self.dB = dA, dB
        self.lam = torch.zeros(M, dtype=torch.float64, device=dev)
        ncols = M if k is None else k
        self.Y = torch.zeros((max(ncols, 1), M), dtype=torch.float64, device=dev)  # column-major
        self.info = torch.full((1,), 777, dtype=torch.int32, device=dev)
        if entry == "solve":
            nbytes = L.gep_workspace_size(M, job, prec)
        elif entry == "lowest":
            nbytes = L.gep_workspace_size_lowest(M, k)
        else:
            nbytes = 0
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        self.nbytes = nbytes

    def enqueue(self):
        import torch
        L = _lib()
        M = self.M
        st = P(torch.cuda.current_stream().cuda_stream)
        a, b = P(self.dA.data_ptr()), P(self.dB.data_ptr())
        lam, Y, info = P(self.lam.data_ptr()), P(self.Y.data_ptr()), P(self.info.data_ptr())
        if self.entry == "solve":
            rc = L.gep_solve(M, a, M, b, M, lam, Y, M, self.job, self.prec,
                             P(self.ws.data_ptr()), self.nbytes, info, st)
        elif self.entry == "noalloc":
            rc = L.gep_solve_noalloc(M, a, M, b, M, lam, Y, M, self.job, self.prec, info, st)
        else:
            rc = L.gep_solve_lowest(M, a, M, b, M, self.k, lam, Y, M, P(self.ws.data_ptr()),
                                    self.nbytes, info, st)
        assert rc == 0, (self.entry, rc)

    def outputs(self):
        return self.lam.clone(), self.Y.clone(), int(self.info.item())


CASES = [
    ("solve", 300, 1, 0, None),
    ("solve", 301, 0, 0, None),
    ("solve", 1100, 1, 0, None),
    ("solve", 400, 1, 1, None),
    ("noalloc", 700, 1, 0, None),
    ("lowest", 500, 1, 0, 120),
]


@pytest.mark.parametrize("entry,M,job,prec,k", CASES)
def test_single_solve_graph_replay(gpu, entry, M, job, prec, k):
    import torch
    say(f"[capture] {entry} M={M} job={job} prec={prec} k={k}")
    A, B = synth.banded_pair(M, synth.decay_length(M), 9300 + M)
    dA, dB = to_gpu(A), to_gpu(B)
    c = _Call(entry, dA, dB, job=job, prec=prec, k=k)
    c.enqueue()
    torch.cuda.synchronize()
    lam0, Y0, info0 = c.outputs()
    assert info0 == 0, info0
    # the eager call against the oracle's eigenvalues
    r = oracle.solve(A, B, vectors=False)
    err = np.abs(to_np(lam0) - r.lam).max() / r.norm1
    assert err <= 1e-11, err
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        c.enqueue()  # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            c.enqueue()
    torch.cuda.synchronize()
    for rep in range(3):
        c.lam.zero_()
        c.Y.zero_()
        c.info.fill_(777)
        _ = torch.randn(1000, 1000, device="cuda").sum().item()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        lam, Y, info = c.outputs()
        assert info == 0, (rep, info)
        assert torch.equal(lam, lam0), rep
        if job == 1:
            assert torch.equal(Y, Y0), rep
    say(f"  eager |dlambda|/|A|_1 {err:.1e}; 3 replays bitwise equal to the eager call")
