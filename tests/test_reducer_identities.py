"""The algebra of the two alternative reducers (section 3.1), checked on the CPU
against the oracle's Cholesky-based route, so that the GPU paths built on it
(gep_solve_explicit_inverse, gep_solve_cholfree) rest on identities that hold:

- explicit inverse (ELPA style): with R = L^-1, C = (R A) R^T is the oracle's
  reduced matrix L^-1 A L^-T, and Y = R^T Z its back transformation;
- Cholesky-free (EigenExa style, Eqs. 7-9): with B W = W D,
  A' = D^-1/2 W^T A W D^-1/2 has the pencil's eigenvalues, Y = W D^-1/2 Z is a
  B-orthonormal eigenvector basis, and Z = D^1/2 W^T Y maps the oracle's
  eigenvectors to orthonormal eigenvectors of A'.

numpy's eigh stands in for the SEP solver of the second route (a library step,
as the oracle's own pins use scipy)."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("M", [1, 7, 60, 150])
def test_explicit_inverse_reproduces_the_oracle_reduction(M):
    A, B = synth.banded_pair(M, max(2.0, np.sqrt(M / 8)), 300 + M)
    L, info = oracle.cholesky(B)
    assert info == 0
    C_ref = oracle.reduce(A, L)
    R = np.linalg.solve(L, np.eye(M))          # R = L^-1, lower triangular
    assert np.abs(np.triu(R, 1)).max(initial=0.0) <= 1e-15 * np.abs(R).max()
    C = (R @ A) @ R.T
    n1 = np.abs(A).sum(axis=0).max()
    kappa_L = np.abs(L).sum(axis=0).max() * np.abs(R).sum(axis=0).max()
    assert np.abs(np.tril(C) - np.tril(C_ref)).max() <= 1e-14 * n1 * kappa_L ** 2
    # back transformation: R^T Z equals the oracle's L^-T Z
    Z = np.linalg.eigh(C_ref)[1]
    assert np.abs(R.T @ Z - oracle.back_transform(L, Z)).max() <= 1e-13 * kappa_L


@pytest.mark.parametrize("M", [1, 7, 60, 150])
def test_cholesky_free_route_reproduces_the_oracle_eigenpairs(M):
    A, B = synth.banded_pair(M, max(2.0, np.sqrt(M / 8)), 400 + M)
    r = oracle.solve(A, B)
    n1 = r.norm1
    d, W = np.linalg.eigh(B)                    # B W = W D (Eq. 7)
    assert d.min() > 0.0
    S = W / np.sqrt(d)[None, :]                 # W D^-1/2
    Ap = S.T @ A @ S                            # A' (Eq. 8)
    lam, Z = np.linalg.eigh(Ap)
    Y = S @ Z                                   # Y = W D^-1/2 Z (Eq. 9)
    kappa = d.max() / d.min()
    assert np.abs(lam - r.lam).max() / n1 <= 1e-12
    assert np.abs(Y.T @ B @ Y - np.eye(M)).max() <= 1e-13 * max(1.0, kappa)
    assert (np.abs(A @ Y - B @ Y * lam[None, :]).sum(axis=0).max()
            / (n1 * np.abs(Y).sum(axis=0).max())) <= 1e-13
    # Z = D^1/2 W^T Y applied to the oracle's eigenvectors: orthonormal eigenvectors of A'
    Zo = (np.sqrt(d)[:, None] * W.T) @ r.Y
    assert np.abs(Zo.T @ Zo - np.eye(M)).max() <= 1e-12 * max(1.0, kappa)
    assert np.abs(Ap @ Zo - Zo * r.lam[None, :]).max() <= 1e-12 * n1 * max(1.0, kappa)


def test_cholesky_free_route_detects_an_indefinite_B():
    """An eigenvalue of B that is not positive is exactly what the Cholesky-free
    path reports (info = M + c); the same B stops the oracle's Cholesky at the
    leading minor of order 21 (reported by the solve as M + 21)."""
    M = 40
    A, B = synth.banded_pair(M, 5.0, 79)
    B[20, 20] = -1.0
    assert int((np.linalg.eigvalsh(B) <= 0).sum()) == 1
    _, info = oracle.cholesky(B)
    assert info == 21
