"""GPU parity of the FP64 MFMA GEMM building block (gep_dgemm) against numpy,
covering transposes, ragged edges, unaligned operands and the lower-only mode."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _run(ta, tb, uplo, m, n, k, alpha, beta, off=0, seed=0):
    import torch
    from paper_1504_06443_amd._binding import lib
    rng = np.random.default_rng(seed)
    Ar, Ac = (k, m) if ta else (m, k)
    Br, Bc = (n, k) if tb else (k, n)
    lda, ldb, ldc = Ar + 3, Br + 1, m + 2
    # column-major storage held in torch tensors of shape (cols, ld) (+ offset)
    A = rng.standard_normal((Ac, lda))
    B = rng.standard_normal((Bc, ldb))
    C = rng.standard_normal((n, ldc))
    dA = torch.from_numpy(np.concatenate([np.zeros(off), A.ravel()])).cuda()
    dB = torch.from_numpy(np.concatenate([np.zeros(off), B.ravel()])).cuda()
    dC = torch.from_numpy(C.ravel().copy()).cuda()
    P = lambda t, o=0: ctypes.c_void_p(t.data_ptr() + 8 * o)
    st = lib().gep_dgemm(ta, tb, uplo, m, n, k, alpha, P(dA, off), lda, P(dB, off), ldb, beta,
                         P(dC), ldc, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    out = dC.cpu().numpy().reshape(n, ldc)[:, :m].T
    Am = A[:, :Ar].T
    Bm = B[:, :Br].T
    opA = Am.T if ta else Am
    opB = Bm.T if tb else Bm
    ref = alpha * opA @ opB + beta * C[:, :m].T
    if uplo:
        mask = np.tril(np.ones((m, n), dtype=bool))
        ref = np.where(mask, ref, C[:, :m].T)
    return out, ref, k


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (17, 33, 5), (128, 128, 16), (300, 257, 129),
                                   (64, 700, 1500), (513, 64, 40)])
def test_dgemm_matches_numpy(gpu, ta, tb, m, n, k):
    say(f"[gemm] ta={ta} tb={tb} {m}x{n}x{k}")
    for off in (0, 1):
        out, ref, kk = _run(ta, tb, 0, m, n, k, 1.25, -0.5, off=off)
        assert np.abs(out - ref).max() <= 1e-14 * max(1, kk) * 4


def test_dgemm_lower_only(gpu):
    say("[gemm] lower only")
    out, ref, k = _run(0, 1, 1, 300, 300, 77, -1.0, 1.0)
    assert np.abs(out - ref).max() <= 1e-14 * k * 4
