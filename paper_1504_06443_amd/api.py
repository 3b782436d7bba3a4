"""Torch-facing wrappers around the libgep C ABI (argument marshalling only)."""
from __future__ import annotations

import ctypes

import torch

from ._binding import JOB_VALUES, JOB_VECTORS, PREC_FP64, PREC_MIXED, check, lib

PHASES = ("R1", "R2-4", "S1", "S2", "S3", "S4", "S5", "R5", "F")

_JOBS = {"values": JOB_VALUES, "vectors": JOB_VECTORS, JOB_VALUES: JOB_VALUES,
         JOB_VECTORS: JOB_VECTORS}
_PRECS = {"fp64": PREC_FP64, "mixed": PREC_MIXED, PREC_FP64: PREC_FP64, PREC_MIXED: PREC_MIXED}


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _square(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda or t.dtype != torch.float64 or t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError(f"{name} must be a square float64 CUDA tensor")
    return t.contiguous()


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _info(device) -> torch.Tensor:
    return torch.zeros(1, dtype=torch.int32, device=device)


def _raise_info(info: torch.Tensor, M: int, where: str) -> None:
    v = int(info.item())
    if v == 0:
        return
    if v > M:
        raise torch.linalg.LinAlgError(f"{where}: the leading minor of order {v - M} of B is "
                                       f"not positive definite (info={v})")
    raise torch.linalg.LinAlgError(f"{where}: eigensolver failed to converge (info={v})")


def solve(A: torch.Tensor, B: torch.Tensor, job="vectors", prec="fp64", check_info=True):
    """All eigenpairs of A y = lambda B y.  Returns (lam, Y) with Y^T B Y = I
    (Y is None for job='values')."""
    A = _square(A, "A")
    B = _square(B, "B")
    M = A.shape[0]
    j = _JOBS[job]
    p = _PRECS[prec]
    dev = A.device
    lam = torch.empty(M, dtype=torch.float64, device=dev)
    Ycm = torch.empty((M, M), dtype=torch.float64, device=dev) if j == JOB_VECTORS else None
    ws_bytes = lib().gep_workspace_size(M, j, p)
    ws = _workspace(ws_bytes, dev)
    info = _info(dev)
    st = lib().gep_solve(M, _ptr(A), max(M, 1), _ptr(B), max(M, 1), _ptr(lam), _ptr(Ycm),
                         max(M, 1), j, p, _ptr(ws), ws.numel(), _ptr(info), _stream())
    check(st, "gep_solve")
    if check_info:
        _raise_info(info, M, "gep_solve")
    return lam, (Ycm.t() if Ycm is not None else None)


def reduce(A: torch.Tensor, B: torch.Tensor, check_info=True):
    """Reducer: (L, C) with B = L L^T and C = L^{-1} A L^{-T}."""
    A = _square(A, "A")
    B = _square(B, "B")
    M = A.shape[0]
    dev = A.device
    Lcm = torch.empty((M, M), dtype=torch.float64, device=dev)
    C = torch.empty((M, M), dtype=torch.float64, device=dev)
    ws = _workspace(lib().gep_reduce_workspace_size(M), dev)
    info = _info(dev)
    st = lib().gep_reduce(M, _ptr(A), max(M, 1), _ptr(B), max(M, 1), _ptr(Lcm), max(M, 1),
                          _ptr(C), max(M, 1), _ptr(ws), ws.numel(), _ptr(info), _stream())
    check(st, "gep_reduce")
    if check_info:
        _raise_info(info, M, "gep_reduce")
    return Lcm.t(), C


def band_reduce(C: torch.Tensor, band_width: int = 0):
    """First reduction stage.  Returns the band in lower band storage as a
    (b+1) x M tensor whose row d holds the d-th subdiagonal."""
    C = _square(C, "C")
    M = C.shape[0]
    dev = C.device
    b = band_width
    if b == 0:
        b = 64 if M >= 2048 else (32 if M >= 256 else 16)
    band = torch.empty((M, b + 1), dtype=torch.float64, device=dev)  # column-major (b+1) x M
    ws = _workspace(lib().gep_band_reduce_workspace_size(M, band_width), dev)
    st = lib().gep_band_reduce(M, _ptr(C), max(M, 1), band_width, _ptr(band), b + 1, _ptr(ws),
                               ws.numel(), _stream())
    check(st, "gep_band_reduce")
    return band.t()


def tridiagonalize(C: torch.Tensor, band_width: int = 0):
    """Both reduction stages: returns (d, e) of a tridiagonal similar to C."""
    C = _square(C, "C")
    M = C.shape[0]
    dev = C.device
    d = torch.empty(M, dtype=torch.float64, device=dev)
    e = torch.empty(max(M - 1, 1), dtype=torch.float64, device=dev)
    ws = _workspace(lib().gep_tridiagonalize_workspace_size(M, band_width), dev)
    st = lib().gep_tridiagonalize(M, _ptr(C), max(M, 1), band_width, _ptr(d), _ptr(e), _ptr(ws),
                                  ws.numel(), _stream())
    check(st, "gep_tridiagonalize")
    return d, e[: max(M - 1, 0)]


def tridiag_eig(d: torch.Tensor, e: torch.Tensor, job="vectors", check_info=True):
    """Eigenvalues (ascending) and, for job='vectors', orthonormal eigenvectors of
    the symmetric tridiagonal (d, e)."""
    d = d.contiguous()
    M = d.numel()
    e = e.contiguous() if e.numel() > 0 else torch.zeros(1, dtype=torch.float64, device=d.device)
    j = _JOBS[job]
    dev = d.device
    lam = torch.empty(M, dtype=torch.float64, device=dev)
    Zcm = torch.empty((M, M), dtype=torch.float64, device=dev) if j == JOB_VECTORS else None
    ws = _workspace(lib().gep_tridiag_eig_workspace_size(M, j), dev)
    info = _info(dev)
    st = lib().gep_tridiag_eig(M, _ptr(d), _ptr(e), _ptr(lam), _ptr(Zcm), max(M, 1), j, _ptr(ws),
                               ws.numel(), _ptr(info), _stream())
    check(st, "gep_tridiag_eig")
    if check_info:
        _raise_info(info, M, "gep_tridiag_eig")
    return lam, (Zcm.t() if Zcm is not None else None)


def dgemm(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None, alpha=1.0, beta=0.0,
          lower_only=False):
    """C = alpha A B + beta C on libgep's FP64 MFMA GEMM (row-major torch views are
    handled as transposed column-major operands)."""
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    A = A.contiguous()
    B = B.contiguous()
    if C is None:
        C = torch.zeros((m, n), dtype=torch.float64, device=A.device)
    assert C.is_contiguous()
    # row-major C = A B  <=>  column-major C^T = B^T A^T
    st = lib().gep_dgemm(0, 0, 1 if lower_only else 0, n, m, k, float(alpha), _ptr(B), max(n, 1),
                         _ptr(A), max(k, 1), float(beta), _ptr(C), max(n, 1), _stream())
    check(st, "gep_dgemm")
    return C


def profile_enable(on: bool = True) -> None:
    lib().gep_profile_enable(1 if on else 0)


def profile_read() -> dict:
    buf = (ctypes.c_double * len(PHASES))()
    n = lib().gep_profile_read(ctypes.cast(buf, ctypes.c_void_p), len(PHASES))
    return {PHASES[i]: buf[i] for i in range(n)}


def solve_batched(As, Bs, job="vectors", prec="fp64", check_info=True):
    raise NotImplementedError("gep_solve_batched is not built yet")


def backward(lam, Y, lam_bar, Y_bar, eta=0.0):
    raise NotImplementedError("gep_backward is not built yet")


class GEPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B):
        raise NotImplementedError("gep_backward is not built yet")
