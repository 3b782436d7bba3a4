"""Helpers shared by the GPU parity tests (comparison metrics only; no solver
arithmetic)."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_gpu(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def to_np(t):
    return t.detach().cpu().numpy()


def clusters(lam, tol):
    """Maximal runs of sorted eigenvalues whose consecutive gaps are <= tol."""
    out = []
    start = 0
    for i in range(1, len(lam) + 1):
        if i == len(lam) or lam[i] - lam[i - 1] > tol:
            out.append((start, i))
            start = i
    return out


def max_subspace_sine(Y, Yref, B, lam_ref, tol):
    """Largest B-sine of the angle between the eigenspaces of each cluster, scaled
    by the cluster's gap to the rest of the spectrum: returns max over clusters of
    sin(angle) * gap.  The sines are the singular values of L^T R with B = L L^T
    and R = Y_S - Yref_S (Yref_S^T B Y_S), the B-orthogonal projection residual
    (computed directly, not from the cosines, which would lose half the digits)."""
    worst = 0.0
    n = len(lam_ref)
    BY = B @ Y
    LB = np.linalg.cholesky(B)
    for a, b in clusters(lam_ref, tol):
        R = Y[:, a:b] - Yref[:, a:b] @ (Yref[:, a:b].T @ BY[:, a:b])
        sin = np.linalg.norm(LB.T @ R, 2)
        gl = lam_ref[a] - lam_ref[a - 1] if a > 0 else np.inf
        gr = lam_ref[b] - lam_ref[b - 1] if b < n else np.inf
        gap = min(gl, gr)
        if np.isfinite(gap):
            worst = max(worst, sin * gap)
    return worst
