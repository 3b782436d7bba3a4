"""GPU parity tests of the solver's phases against the CPU oracle, through the
C ABI (via the thin Python binding)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import say, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _gep():
    import paper_1504_06443_amd as gep
    return gep


@pytest.mark.parametrize("M", [1, 2, 5, 64, 127, 128, 129, 300, 513])
def test_reduce_matches_oracle(gpu, M):
    say(f"[reduce] M={M}")
    A, B = synth.banded_pair(M, max(2.0, M / 40), 200 + M)
    L, C = _gep().reduce(to_gpu(A), to_gpu(B))
    L = to_np(L)
    C = to_np(C)
    Lo, info = oracle.cholesky(B)
    assert info == 0
    Co = oracle.reduce(A, Lo)
    assert np.abs(np.triu(L, 1)).max() == 0.0
    assert np.abs(L - Lo).max() <= 1e-14 * 16
    n1 = oracle.norm1_sym_lower(A)
    assert np.abs(C - Co).max() <= 1e-13 * n1


def test_reduce_reports_indefinite_B(gpu):
    say("[reduce] indefinite B")
    M = 200
    A, B = synth.banded_pair(M, 5.0, 7)
    B[150, 150] = -2.0
    import torch
    gep = _gep()
    with pytest.raises(torch.linalg.LinAlgError) as ei:
        gep.reduce(to_gpu(A), to_gpu(B))
    assert "151" in str(ei.value) or "info=351" in str(ei.value)


def _band_to_dense(band, M):
    b = band.shape[0] - 1
    T = np.zeros((M, M))
    for d in range(b + 1):
        for j in range(M - d):
            T[j + d, j] = band[d, j]
            T[j, j + d] = band[d, j]
    return T


@pytest.mark.parametrize("M,b", [(3, 16), (40, 16), (100, 16), (300, 32), (333, 64), (700, 64)])
def test_band_reduce_preserves_spectrum(gpu, M, b):
    say(f"[band] M={M} b={b}")
    A, B = synth.banded_pair(M, 6.0, 300 + M)
    Lo, _ = oracle.cholesky(B)
    C = oracle.reduce(A, Lo)
    band = to_np(_gep().band_reduce(to_gpu(C), b))
    T = _band_to_dense(band, M)
    w_ref = oracle.tridiag_eigvals(*oracle.tridiagonalize(C)[:2])
    w_band = oracle.tridiag_eigvals(*oracle.tridiagonalize(T)[:2])
    scale = np.abs(C).sum(axis=0).max()
    assert np.abs(w_band - w_ref).max() <= 1e-13 * scale
    assert abs(np.linalg.norm(T) - np.linalg.norm(C)) <= 1e-13 * np.linalg.norm(C)


def test_band_reduce_split_symm(gpu):
    """M = 2150, b = 64: the first panel's trailing product A22 V has 2086 >= 2048
    rows, so it splits K (the symmetric operand read through its mirror with
    absolute k).  The band's eigenvalues come from LAPACK's banded symmetric
    eigensolver (a library step on the test side); the reference is the oracle's."""
    import scipy.linalg
    M, b = 2150, 64
    say(f"[band] split SYMM M={M} b={b}")
    A, B = synth.banded_pair(M, 6.0, 300 + M)
    Lo, _ = oracle.cholesky(B)
    C = oracle.reduce(A, Lo)
    band = to_np(_gep().band_reduce(to_gpu(C), b))
    w_ref = oracle.tridiag_eigvals(*oracle.tridiagonalize(C)[:2])
    w_band = np.sort(scipy.linalg.eigvals_banded(band, lower=True))
    scale = np.abs(C).sum(axis=0).max()
    assert np.abs(w_band - w_ref).max() <= 1e-13 * scale
    fro_band = np.sqrt((band[0] ** 2).sum() + 2 * (band[1:] ** 2).sum())
    assert abs(fro_band - np.linalg.norm(C)) <= 1e-13 * np.linalg.norm(C)


@pytest.mark.parametrize("M,b", [(2, 16), (3, 16), (50, 16), (257, 32), (700, 64), (1100, 64)])
def test_tridiagonalize_preserves_spectrum(gpu, M, b):
    say(f"[tridiag] M={M} b={b}")
    A, B = synth.banded_pair(M, 8.0, 400 + M)
    Lo, _ = oracle.cholesky(B)
    C = oracle.reduce(A, Lo)
    d, e = _gep().tridiagonalize(to_gpu(C), b)
    d, e = to_np(d), to_np(e)
    w_ref = oracle.tridiag_eigvals(*oracle.tridiagonalize(C)[:2])
    w = oracle.tridiag_eigvals(d, e)
    scale = np.abs(C).sum(axis=0).max()
    assert np.abs(w - w_ref).max() <= 1e-13 * scale
    fro = np.sqrt((d ** 2).sum() + 2 * (e ** 2).sum())
    assert abs(fro - np.linalg.norm(C)) <= 1e-13 * np.linalg.norm(C)


def _tridiag_cases():
    rng = np.random.default_rng(9)
    cases = []
    for M in (1, 2, 3, 64, 65, 200, 1000):
        cases.append((f"random{M}", rng.standard_normal(M), rng.standard_normal(max(M - 1, 0))))
    for M in (97, 512):
        cases.append((f"toeplitz{M}", np.full(M, 0.3), np.full(M - 1, -1.1)))
    M = 300
    i = np.arange(1, M)
    cases.append(("clement300", np.zeros(M), np.sqrt(i * (M - i)).astype(float)))
    # glued Wilkinson matrices: tight clusters, heavy deflation
    W = np.abs(np.arange(-10, 11)).astype(float)
    d = np.concatenate([W] * 20)
    e = np.ones(d.size - 1)
    e[20::21] = 1e-9
    cases.append(("glued_wilkinson", d, e))
    # zero couplings (splits) and repeated values
    d = np.repeat(np.arange(5.0), 40)
    e = np.zeros(199)
    cases.append(("diagonal_repeated", d, e))
    return cases


@pytest.mark.parametrize("M", [8192, 8195])
def test_tridiag_eig_large_matches_oracle(gpu, M):
    """Orders >= 8192 run the top three merge levels' GEMMs with host-side sizes
    on the tiled GEMM path.  An even order takes the fast kernel (with the bottom
    product shifted by one zero column when the top half's undeflated count is
    odd); an odd order (odd leading dimension) takes the grouped fallback."""
    say(f"[stedc] large random M={M}")
    rng = np.random.default_rng(11 + M)
    d, e = rng.standard_normal(M), rng.standard_normal(M - 1)
    lam, Z = _gep().tridiag_eig(to_gpu(d), to_gpu(e))
    lam, Z = to_np(lam), to_np(Z)
    w_ref = oracle.tridiag_eigvals(d, e)
    tn = np.abs(d).max() + 2 * np.abs(e).max()
    assert np.all(np.diff(lam) >= 0)
    assert np.abs(lam - w_ref).max() <= 1e-13 * tn * 4
    assert np.abs(Z.T @ Z - np.eye(M)).max() <= 1e-13 * np.sqrt(M)
    TZ = d[:, None] * Z
    TZ[1:] += e[:, None] * Z[:-1]
    TZ[:-1] += e[:, None] * Z[1:]
    assert np.abs(TZ - Z * lam[None, :]).max() <= 1e-13 * tn * np.sqrt(M)


@pytest.mark.parametrize("name,d,e", _tridiag_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_tridiag_eig_matches_oracle(gpu, name, d, e):
    say(f"[stedc] {name} M={d.size}")
    M = d.size
    lam, Z = _gep().tridiag_eig(to_gpu(d), to_gpu(e))
    lam, Z = to_np(lam), to_np(Z)
    w_ref = oracle.tridiag_eigvals(d, e)
    tn = np.abs(d).max() + 2 * (np.abs(e).max() if e.size else 0.0)
    assert np.all(np.diff(lam) >= 0)
    assert np.abs(lam - w_ref).max() <= 1e-13 * max(tn, 1.0) * 4
    T = np.diag(d) + np.diag(e, -1) + np.diag(e, 1)
    assert np.abs(Z.T @ Z - np.eye(M)).max() <= 1e-13 * max(8, np.sqrt(M))
    assert np.abs(T @ Z - Z * lam[None, :]).max() <= 1e-13 * max(tn, 1.0) * max(8, np.sqrt(M))
    lam_b, _ = _gep().tridiag_eig(to_gpu(d), to_gpu(e), job="values")
    assert np.abs(to_np(lam_b) - w_ref).max() <= 1e-13 * max(tn, 1.0) * 4
