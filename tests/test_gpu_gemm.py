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
                         P(dC), ldc, 0, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
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


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_fp32_arithmetic(gpu, ta, tb):
    """arith = 1: interior tiles multiply FP32-rounded operands with FP32
    accumulation.  Bound: |C - fl32(A) fl32(B)| <= gamma_k |fl32(A)| |fl32(B)|
    elementwise, gamma_k = k u / (1 - k u), u = 2^-24 (standard dot-product error
    bound); the FP64 edge strips meet it trivially."""
    import torch
    from paper_1504_06443_amd._binding import lib
    rng = np.random.default_rng(11 + 2 * ta + tb)
    m, n, k = 1100, 1800, 520  # >= 128 tiles of 128 x 128: interior kernel + strips
    Ar, Ac = (k, m) if ta else (m, k)
    Br, Bc = (n, k) if tb else (k, n)
    A = rng.standard_normal((Ac, Ar))   # column-major Ar x Ac held as rows of length Ar
    B = rng.standard_normal((Bc, Br))
    dA, dB = torch.from_numpy(A.ravel().copy()).cuda(), torch.from_numpy(B.ravel().copy()).cuda()
    dC = torch.zeros(n * m, dtype=torch.float64, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    st = lib().gep_dgemm(ta, tb, 0, m, n, k, 1.0, P(dA), Ar, P(dB), Br, 0.0, P(dC), m, 1,
                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    out = dC.cpu().numpy().reshape(n, m).T
    A32 = A.astype(np.float32).astype(np.float64).T
    B32 = B.astype(np.float32).astype(np.float64).T
    opA = A32.T if ta else A32
    opB = B32.T if tb else B32
    ref = opA @ opB
    u = 2.0 ** -24
    gamma = k * u / (1 - k * u)
    bound = gamma * (np.abs(opA) @ np.abs(opB))
    assert np.all(np.abs(out - ref) <= bound)
    # and it is not FP64 arithmetic on the interior: the error is FP32-sized there
    assert np.abs(out - ref)[:1024, :1792].max() > 1e-10
    # the bottom strip stays FP64 on the unrounded operands
    A64, B64 = A.T, B.T
    ref64 = (A64.T if ta else A64) @ (B64.T if tb else B64)
    assert np.abs(out - ref64)[1024:, :].max() <= 1e-12 * np.abs(ref64).max()


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("alpha,beta", [(-1.0, 1.0), (1.0, 0.5), (-1.0, -2.0), (1.25, -0.5)])
def test_dgemm_interior_kernel(gpu, ta, tb, alpha, beta):
    """Shapes with >= 128 tiles of 128 x 128 run the interior kernel (plus k tail
    and edge strips); alpha = +-1 with beta != 0 takes the path that starts the
    accumulators from alpha beta C, the others the FP64 epilogue."""
    say(f"[gemm] interior ta={ta} tb={tb} alpha={alpha} beta={beta}")
    out, ref, kk = _run(ta, tb, 0, 1100, 1800, 520, alpha, beta, seed=3)
    assert np.abs(out - ref).max() <= 1e-14 * kk * 4 * max(1.0, abs(beta))


@pytest.mark.parametrize("alpha,beta", [(-1.0, 1.0), (1.0, 0.0)])
def test_dgemm_interior_lower_only(gpu, alpha, beta):
    say(f"[gemm] interior lower alpha={alpha} beta={beta}")
    out, ref, k = _run(0, 1, 1, 1664, 1664, 256, alpha, beta, seed=4)
    assert np.abs(out - ref).max() <= 1e-14 * k * 4
