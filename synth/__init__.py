"""Seeded synthetic inputs for the dense generalized symmetric-definite eigenproblem.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds no
step of the eigensolver: it only draws random matrices.  The paper measures on
tight-binding Hamiltonian/overlap pairs (H = A, S = B) from the ELSES matrix
library (section 2.2); those files are not available here, so the generator below
stands in for them: a Hamiltonian whose entries decay with |i - j| (local
orbitals), and an overlap matrix close to the identity with the same decay.

Recipe (all FP64):

* ``D_ij = exp(-|i - j| / ell)``.
* ``X_ij = D_ij * g_ij`` with ``g ~ N(0, 1)``; ``A = (X + X^T) / 2``; then the
  diagonal is overwritten with ``A_ii ~ U(-10, 0)``.
* ``W_ij = D_ij * h_ij`` (``h ~ N(0, 1)``), ``W_ii = 0``; ``S = W + W^T``;
  ``s = 0.5 / max_i sum_j |S_ij|``; ``B = I + s * S``.  Gershgorin then puts the
  spectrum of B inside [0.5, 1.5], so B is SPD with condition number <= 3.
* Random streams: row block ``r`` (``ROWS`` rows) of ``g`` is drawn from
  ``default_rng([seed, 0, r])``, the diagonal from ``default_rng([seed, 1])``,
  row block ``r`` of ``h`` from ``default_rng([seed, 2, r])``.  Row blocks are
  independent streams so the large cases can be drawn by several threads and
  still be bit-identical on every machine.

A symmetric matrix has the same bytes in row- and column-major order, so the
arrays returned here can be handed to column-major code unchanged.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROWS = 512


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _decayed_normals(M: int, ell: float, seed: int, tag: int) -> np.ndarray:
    out = np.empty((M, M), dtype=np.float64)
    cols = np.arange(M, dtype=np.float64)

    def fill(r: int) -> None:
        lo, hi = r * ROWS, min(M, (r + 1) * ROWS)
        rng = np.random.default_rng([seed, tag, r])
        blk = out[lo:hi]
        rng.standard_normal(out=blk)
        rows = np.arange(lo, hi, dtype=np.float64)[:, None]
        blk *= np.exp(-np.abs(rows - cols[None, :]) / ell)

    nblk = (M + ROWS - 1) // ROWS
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(fill, range(nblk)))
    return out


def _symmetrize_inplace(X: np.ndarray, scale: float) -> None:
    """X <- scale * (X + X^T), block by block, without a second M x M buffer."""
    M = X.shape[0]
    nb = 1024
    starts = list(range(0, M, nb))

    def row(I: int) -> None:
        i0, i1 = I, min(M, I + nb)
        for J in starts:
            if J > I:
                break
            j0, j1 = J, min(M, J + nb)
            a = X[i0:i1, j0:j1]
            b = X[j0:j1, i0:i1]
            s = scale * (a + b.T)
            X[i0:i1, j0:j1] = s
            X[j0:j1, i0:i1] = s.T

    # Block rows touch disjoint (I, J) / (J, I) pairs, so they run in parallel.
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(row, starts))


def decay_length(M: int) -> float:
    """Decay length used where a case does not fix one: sqrt(M / 8).

    It gives 8, 32 and 64 for M = 512, 8192 and 32768."""
    return math.sqrt(M / 8.0)


def hamiltonian(M: int, ell: float, seed: int) -> np.ndarray:
    A = _decayed_normals(M, ell, seed, 0)
    _symmetrize_inplace(A, 0.5)
    A[np.diag_indices(M)] = np.random.default_rng([seed, 1]).uniform(-10.0, 0.0, M)
    return A


def overlap(M: int, ell: float, seed: int) -> np.ndarray:
    W = _decayed_normals(M, ell, seed, 2)
    W[np.diag_indices(M)] = 0.0
    _symmetrize_inplace(W, 1.0)  # W <- W + W^T
    rowsum = np.empty(M)
    for i0 in range(0, M, 4096):
        rowsum[i0:i0 + 4096] = np.abs(W[i0:i0 + 4096]).sum(axis=1)
    s = 0.5 / rowsum.max() if rowsum.max() > 0 else 0.0
    W *= s
    W[np.diag_indices(M)] += 1.0
    return W


def banded_pair(M: int, ell: float | None = None, seed: int = 0):
    """(A, B) for one generalized eigenproblem of order M."""
    if ell is None:
        ell = decay_length(M)
    return hamiltonian(M, ell, seed), overlap(M, ell, seed)


# Named workloads -----------------------------------------------------------

#: (M, decay length, seed) of the single-problem workloads.
SINGLE = {
    "m512": (512, 8.0, 1),
    "m8192": (8192, 32.0, 2),
    "m32768": (32768, 64.0, 3),
    "m4096_grad": (4096, decay_length(4096), 5),
}


def workload(name: str):
    M, ell, seed = SINGLE[name]
    return banded_pair(M, ell, seed)


def batch_sizes(count: int = 256, lo: int = 64, hi: int = 2048, seed: int = 4) -> list[int]:
    """Orders drawn log-uniformly in [lo, hi]."""
    u = np.random.default_rng(seed).uniform(math.log(lo), math.log(hi), count)
    return [int(min(hi, max(lo, round(math.exp(x))))) for x in u]


def batch_instance(i: int, M: int):
    """Instance i of the batch: its own seed, decay length sqrt(M/8)."""
    return banded_pair(M, decay_length(M), 4000 + i)


def symmetric_normal(M: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Symmetric matrix whose upper triangle (diagonal included) is i.i.d.
    N(0, scale^2), mirrored into the lower triangle."""
    g = np.random.default_rng(seed).standard_normal((M, M)) * scale
    U = np.triu(g)
    return U + np.triu(U, 1).T


def unit_direction(M: int, seed: int) -> np.ndarray:
    """Symmetric N(0,1) direction scaled to unit Frobenius norm."""
    E = symmetric_normal(M, seed)
    return E / np.linalg.norm(E)


def probe_matrix(M: int, k: int, seed: int) -> np.ndarray:
    """M x k i.i.d. N(0,1) probe vectors (random projections for comparing large
    matrices through a few products)."""
    return np.random.default_rng(seed).standard_normal((M, k))


def sample_pairs(M: int, count: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """`count` uniformly drawn (row, column) index pairs of an M x M matrix."""
    g = np.random.default_rng(seed)
    return g.integers(0, M, count), g.integers(0, M, count)


def toeplitz_tridiag(M: int, a: float, b: float) -> np.ndarray:
    T = np.zeros((M, M))
    T[np.diag_indices(M)] = a
    i = np.arange(M - 1)
    T[i + 1, i] = b
    T[i, i + 1] = b
    return T
