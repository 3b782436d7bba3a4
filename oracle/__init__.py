"""CPU oracle for the dense generalized symmetric-definite eigenproblem.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library.  It shares no code with
the GPU path (``liboracle.so`` is built from ``oracle/oracle.c`` alone).

What it computes (the plain definition of the method's result):

* the eigenvalues of the pencil (A, B), ascending, and a B-orthonormal set of
  eigenvectors Y with ``A Y = B Y Lambda`` and ``Y^T B Y = I`` (section 1, Eq. 1;
  section 3.1, Eq. 2);
* along the way the unique intermediates of the reducer: the Cholesky factor
  ``B = L L^T`` (Eq. 4, with L = U^T) and the reduced matrix ``C = L^{-1} A L^{-T}``
  (Eq. 5), and the back transformation ``Y = L^{-T} Z`` (Eq. 6);
* the adjoint of the eigen-decomposition (``gradient``), obtained by
  differentiating ``A Y = B Y Lambda`` and ``Y^T B Y = I``.

Sign convention for eigenvectors: the entry of largest magnitude in each column
is positive (the lowest index wins a tie).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

BUILD_CMD = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", _SRC, "-o", _LIB_PATH, "-lm"]


def build(force: bool = True) -> str:
    """Compile liboracle.so from oracle.c with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(BUILD_CMD)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        D = ctypes.c_double
        L.orc_threads.restype = ctypes.c_int
        L.orc_cholesky.argtypes = [I, P, I]
        L.orc_cholesky.restype = I
        L.orc_reduce.argtypes = [I, P, I, P, I, P]
        L.orc_reduce.restype = None
        L.orc_back_transform.argtypes = [I, I, P, I, P, I]
        L.orc_back_transform.restype = None
        L.orc_tridiagonalize.argtypes = [I, P, P, P, P]
        L.orc_tridiagonalize.restype = None
        L.orc_form_q.argtypes = [I, P, P, P]
        L.orc_form_q.restype = None
        L.orc_sturm_count.argtypes = [I, P, P, D]
        L.orc_sturm_count.restype = I
        L.orc_bisect_all.argtypes = [I, P, P, P]
        L.orc_bisect_all.restype = None
        L.orc_tql.argtypes = [I, P, P, P, I]
        L.orc_tql.restype = I
        L.orc_ldlt_inertia.argtypes = [I, P, I]
        L.orc_ldlt_inertia.restype = I
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().orc_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64F(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


# --- steps -------------------------------------------------------------------

def cholesky(B):
    """L with B = L L^T (lower triangle of B read).  Returns (L, info); info = k > 0
    if the leading minor of order k is not positive definite (Eq. 4)."""
    L = _f64F(B).copy(order="F")
    n = L.shape[0]
    info = lib().orc_cholesky(n, _ptr(L), n)
    return L, int(info)


def reduce(A, L):
    """C = L^{-1} A L^{-T} by forward substitutions (Eq. 5)."""
    A = _f64F(A)
    L = _f64F(L)
    n = A.shape[0]
    C = np.empty((n, n), order="F")
    lib().orc_reduce(n, _ptr(A), n, _ptr(L), n, _ptr(C))
    return C


def back_transform(L, Z):
    """Y = L^{-T} Z by back substitution (Eq. 6)."""
    L = _f64F(L)
    Y = _f64F(Z).copy(order="F")
    n, k = Y.shape
    lib().orc_back_transform(n, k, _ptr(L), n, _ptr(Y), n)
    return Y


def tridiagonalize(C):
    """One-stage Householder reduction C = Q T Q^T.  Returns (d, e, refl, beta)
    where refl holds the reflectors below the subdiagonal."""
    R = _f64F(C).copy(order="F")
    n = R.shape[0]
    d = np.empty(n)
    e = np.empty(max(n - 1, 1))
    beta = np.zeros(max(n, 1))
    lib().orc_tridiagonalize(n, _ptr(R), _ptr(d), _ptr(e), _ptr(beta))
    return d, e[: max(n - 1, 0)], R, beta


def form_q(refl, beta):
    n = refl.shape[0]
    Q = np.empty((n, n), order="F")
    lib().orc_form_q(n, _ptr(_f64F(refl)), _ptr(np.ascontiguousarray(beta, dtype=np.float64)), _ptr(Q))
    return Q


def sturm_count(d, e, x: float) -> int:
    """Number of eigenvalues of the tridiagonal (d, e) below x."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    if e.size == 0:
        e = np.zeros(1)
    return int(lib().orc_sturm_count(d.size, _ptr(d), _ptr(e), float(x)))


def tridiag_eigvals(d, e):
    """All eigenvalues of the tridiagonal (d, e), ascending, by Sturm bisection."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = d.size
    if n == 0:
        return np.empty(0)
    if e.size == 0:
        e = np.zeros(1)
    w = np.empty(n)
    lib().orc_bisect_all(n, _ptr(d), _ptr(e), _ptr(w))
    return w


def tql(d, e, Z):
    """Implicit QL on (d, e) accumulating rotations into Z.  Returns (w, Z, info),
    w unordered."""
    dd = np.ascontiguousarray(d, dtype=np.float64).copy()
    n = dd.size
    ee = np.zeros(max(n, 1))
    ee[: n - 1] = np.asarray(e, dtype=np.float64)[: n - 1]
    Z = _f64F(Z).copy(order="F")
    info = lib().orc_tql(n, _ptr(dd), _ptr(ee), _ptr(Z), Z.shape[0])
    return dd, Z, int(info)


def sign_fix(Y: np.ndarray) -> np.ndarray:
    """Make the entry of largest magnitude in each column positive."""
    if Y.size == 0:
        return Y
    idx = np.argmax(np.abs(Y), axis=0)
    s = np.sign(Y[idx, np.arange(Y.shape[1])])
    s[s == 0] = 1.0
    return Y * s[None, :]


# --- whole problem -----------------------------------------------------------

class OracleResult:
    def __init__(self, lam, Y, info, L=None, C=None, d=None, e=None, norm1=None):
        self.lam = lam
        self.Y = Y
        self.info = info
        self.L = L
        self.C = C
        self.d = d
        self.e = e
        self.norm1 = norm1


def norm1_sym_lower(A) -> float:
    """||A||_1 (max column sum) of the symmetric matrix whose lower triangle is A."""
    A = np.asarray(A, dtype=np.float64)
    S = np.tril(A) + np.tril(A, -1).T
    return float(np.abs(S).sum(axis=0).max()) if S.size else 0.0


def solve(A, B, vectors: bool = True, keep: bool = False) -> OracleResult:
    """All eigenpairs of A y = lambda B y.

    Steps: Cholesky (Eq. 4); C = L^{-1} A L^{-T} (Eq. 5); tridiagonalise C;
    eigenvalues by bisection; if vectors: implicit QL accumulated on Q, then
    Y = L^{-T} Z (Eq. 6); sort ascending; sign convention.
    info follows the LAPACK generalized-driver convention: M + k when the leading
    minor k of B is not positive definite, k when the QL iteration failed at k.
    """
    A = _f64F(A)
    B = _f64F(B)
    n = A.shape[0]
    if n == 0:
        return OracleResult(np.empty(0), np.empty((0, 0)), 0)
    L, info = cholesky(B)
    if info:
        return OracleResult(None, None, n + info)
    C = reduce(A, L)
    d, e, refl, beta = tridiagonalize(C)
    lam = tridiag_eigvals(d, e)
    Y = None
    info = 0
    if vectors:
        Q = form_q(refl, beta)
        w, Z, info = tql(d, e, Q)
        Y = back_transform(L, Z)
        order = np.argsort(w, kind="stable")
        Y = sign_fix(Y[:, order])
    return OracleResult(lam, Y, info, L if keep else None, C if keep else None,
                        d if keep else None, e if keep else None, norm1_sym_lower(A))


def inertia_count(A, B, sigma: float) -> int:
    """Number of eigenvalues of the pencil (A, B) below sigma, without solving it.

    B is positive definite, so A - sigma B is congruent to C - sigma I with
    C = L^{-1} A L^{-T} (Eq. 5), and by Sylvester's law of inertia the number of
    negative eigenvalues of A - sigma B is #{lambda_k < sigma}.  That number is
    read off a symmetric indefinite factorisation of A - sigma B with diagonal
    pivoting (orc_ldlt_inertia: Bunch-Kaufman, plain C) as the number of negative
    eigenvalues of its block-diagonal factor.  Only the lower triangles of A and
    B are read.  Raises ValueError when a pivot is exactly singular (sigma is an
    eigenvalue).
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    n = A.shape[0]
    if n == 0:
        return 0
    # lower triangle of A - sigma B, built column block by column block in
    # Fortran order (symmetric inputs: the transpose view of C-ordered data)
    W = np.empty((n, n), order="F")
    step = 2048
    for j0 in range(0, n, step):
        j1 = min(n, j0 + step)
        W[:, j0:j1] = np.tril(A[:, j0:j1], -j0) - sigma * np.tril(B[:, j0:j1], -j0)
    neg = int(lib().orc_ldlt_inertia(n, _ptr(W), n))
    if neg < 0:
        raise ValueError("A - sigma B is singular: sigma is an eigenvalue")
    return neg


def eigvals(A, B) -> np.ndarray:
    return solve(A, B, vectors=False).lam


# --- adjoint -----------------------------------------------------------------

def gradient(lam, Y, lam_bar=None, Y_bar=None, eta: float = 0.0, tau_c: float = 0.0):
    """Adjoint of (lambda, Y) = eig(A, B) for symmetric perturbations.

    Differentiating A Y = B Y Lambda and Y^T B Y = I with P = Y^T dA Y and
    Q = Y^T dB Y gives d lambda_i = P_ii - lambda_i Q_ii and dY = Y Omega with
    Omega_ij = (P_ij - lambda_j Q_ij)/(lambda_j - lambda_i) (i != j),
    Omega_ii = -Q_ii / 2.  Transposing this linear map:

        Wb   = Y^T Y_bar,  Wa = (Wb - Wb^T)/2,  Ws = (Wb + Wb^T)/2
        F_ij = D / (D^2 + eta^2) with D = lambda_j - lambda_i, F = 0 if |D| <= tau_c
        Pb   = F o Wa + diag(lambda_bar)
        A_bar = Y Pb Y^T
        B_bar = -1/2 Y (Lambda Pb + Pb Lambda + Ws) Y^T

    For losses that are invariant under rotations inside a degenerate eigenspace,
    zeroing F inside the degenerate set is exact.  Returns symmetric (A_bar, B_bar).
    """
    lam = np.asarray(lam, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    M = lam.size
    Pb = np.zeros((M, M))
    Ws = np.zeros((M, M))
    if Y_bar is not None:
        Wb = Y.T @ np.asarray(Y_bar, dtype=np.float64)
        Wa = 0.5 * (Wb - Wb.T)
        Ws = 0.5 * (Wb + Wb.T)
        D = lam[None, :] - lam[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            F = D / (D * D + eta * eta)
        F[np.abs(D) <= tau_c] = 0.0
        np.fill_diagonal(F, 0.0)
        Pb += F * Wa
    if lam_bar is not None:
        Pb[np.diag_indices(M)] += np.asarray(lam_bar, dtype=np.float64)
    Ab = Y @ Pb @ Y.T
    inner = lam[:, None] * Pb + Pb * lam[None, :] + Ws
    Bb = -0.5 * (Y @ inner @ Y.T)
    Ab = 0.5 * (Ab + Ab.T)
    Bb = 0.5 * (Bb + Bb.T)
    return Ab, Bb
