"""GPU parity of the mixed-precision solve (gep_solve with GEP_PREC_MIXED: FP32
arithmetic in the interior GEMM tiles, then one FP64 refinement pass) against the
CPU oracle.  The eigenvalue bar is the FP64 one (|d lambda| / ||A||_1 <= 1e-11);
the refinement corrects the vectors to first order in the coupling c left
between blocks (|c| is FP32 rounding over an eigenvalue gap, about 1e-3 at most
on these matrices), so B-orthogonality and the residual are of order c^2 and are
held to 1e-5 and 1e-7 and printed."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import max_subspace_sine, say, to_gpu, to_np

pytestmark = pytest.mark.gpu

TOL_LAMBDA = 1e-11
TOL_ORTH_MIXED = 1e-5
TOL_RES_MIXED = 1e-7
TOL_SUBSPACE_MIXED = 1e-5


def _gep():
    import paper_1504_06443_amd as gep
    return gep


def _metrics(A, B, lam, Y, r):
    M = A.shape[0]
    n1 = r.norm1
    err = np.abs(lam - r.lam).max() / n1
    orth = np.abs(Y.T @ B @ Y - np.eye(M)).max()
    res = np.abs(A @ Y - B @ Y * lam[None, :]).sum(axis=0).max() / (n1 * np.abs(Y).sum(axis=0).max())
    return err, orth, res


@pytest.mark.parametrize("M", [1, 2, 3, 40, 64, 65, 97, 128, 129, 300, 513, 1000])
def test_mixed_against_oracle(gpu, M):
    say(f"[mixed] M={M}")
    A, B = synth.banded_pair(M, max(2.0, np.sqrt(M / 8)), 700 + M)
    lam, Y = _gep().solve(to_gpu(A), to_gpu(B), prec="mixed")
    lam, Y = to_np(lam), to_np(Y)
    r = oracle.solve(A, B)
    assert np.all(np.diff(lam) >= 0)
    err, orth, res = _metrics(A, B, lam, Y, r)
    # eigenspaces against the oracle's: B-angle sine times the cluster's gap, per
    # cluster (first-order refined vectors: held to 1e-5 |A|_1, printed)
    sine_gap = max_subspace_sine(Y, r.Y, B, r.lam, 1e-8 * r.norm1) if M > 1 else 0.0
    say(f"  err {err:.2e} orth {orth:.2e} res {res:.2e} sin*gap/|A|_1 {sine_gap / r.norm1:.2e}")
    assert err <= TOL_LAMBDA
    assert orth <= TOL_ORTH_MIXED
    assert res <= TOL_RES_MIXED
    assert sine_gap <= TOL_SUBSPACE_MIXED * r.norm1


def test_mixed_c1_workload(gpu):
    say("[mixed] m512 workload")
    A, B = synth.workload("m512")
    lam, Y = _gep().solve(to_gpu(A), to_gpu(B), prec="mixed")
    r = oracle.solve(A, B)
    err, orth, res = _metrics(A, B, to_np(lam), to_np(Y), r)
    say(f"  err {err:.2e} orth {orth:.2e} res {res:.2e}")
    assert err <= TOL_LAMBDA and orth <= TOL_ORTH_MIXED and res <= TOL_RES_MIXED


def test_mixed_total_degeneracy(gpu):
    """A = alpha B: every eigenvalue is alpha, every B-orthonormal basis is an
    eigenbasis; the refinement must neither divide by the zero gaps nor lose
    B-orthogonality."""
    say("[mixed] A = alpha B")
    M = 200
    _, B = synth.banded_pair(M, 5.0, 79)
    lam, Y = _gep().solve(to_gpu(-2.25 * B), to_gpu(B), prec="mixed")
    lam, Y = to_np(lam), to_np(Y)
    assert np.abs(lam + 2.25).max() <= 1e-11 * np.abs(2.25 * B).sum(0).max()
    assert np.abs(Y.T @ B @ Y - np.eye(M)).max() <= TOL_ORTH_MIXED


def test_mixed_prescribed_clusters(gpu):
    """Known spectrum with tight clusters (multiplicities 2..6 at 1e-10 spacing):
    clusters stay inside one refinement block, eigenvalues to 1e-11 ||A||_1."""
    say("[mixed] clusters")
    M = 240
    rng = np.random.default_rng(81)
    _, B = synth.banded_pair(M, 4.0, 82)
    LB = np.linalg.cholesky(B)
    Q, _ = np.linalg.qr(rng.standard_normal((M, M)))
    mu = np.sort(rng.uniform(-5, 5, M))
    for start, mult in [(20, 2), (60, 3), (120, 6), (200, 4)]:
        mu[start:start + mult] = mu[start] + 1e-10 * np.arange(mult)
    A = LB @ Q @ np.diag(mu) @ Q.T @ LB.T
    A = 0.5 * (A + A.T)
    lam, Y = _gep().solve(to_gpu(A), to_gpu(B), prec="mixed")
    lam = to_np(lam)
    n1 = np.abs(A).sum(0).max()
    assert np.abs(lam - np.sort(mu)).max() <= 1e-11 * n1 + 1e-14 * np.abs(mu).max() * 10


def test_mixed_rejects_values_only(gpu):
    import torch
    gep = _gep()
    A, B = synth.banded_pair(10, 2.0, 1)
    with pytest.raises(gep.GEPError):
        gep.solve(to_gpu(A), to_gpu(B), job="values", prec="mixed")


@pytest.mark.parametrize("M", [2113, 3001])
def test_mixed_with_fp32_q2(gpu, M):
    """The mixed path with its Q2 back transformation in FP32 arithmetic (tuning
    parameter q2_mixed_fp32 = 1; the built-in choice is FP64, measured faster):
    the refined eigenpairs must meet the same bars as with the FP64 Q2."""
    import paper_1504_06443_amd as gep
    from paper_1504_06443_amd import _binding
    L = _binding.lib()
    say(f"[mixed] FP32 Q2 M={M}")
    A, B = synth.banded_pair(M, max(2.0, np.sqrt(M / 8)), 900 + M)
    dA, dB = to_gpu(A), to_gpu(B)
    lam64, _ = gep.solve(dA, dB)
    assert L.gep_tune_set(b"q2_mixed_fp32", M, M, 1) == 0
    try:
        lam, Y = gep.solve(dA, dB, prec="mixed")
    finally:
        L.gep_tune_reset_overrides()
    lam, Y, lam64 = to_np(lam), to_np(Y), to_np(lam64)
    n1 = np.abs(A).sum(axis=0).max()
    assert np.abs(lam - lam64).max() <= 1e-11 * n1
    assert np.abs(Y.T @ B @ Y - np.eye(M)).max() <= 1e-5
    res = np.abs(A @ Y - B @ Y * lam[None, :]).sum(axis=0).max() / (n1 * np.abs(Y).sum(axis=0).max())
    assert res <= 1e-7, res
