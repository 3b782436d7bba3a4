"""Torch-facing wrappers around the libgep C ABI (argument marshalling only)."""
from __future__ import annotations

import ctypes

import torch

from ._binding import (INFO_REFINE_FAILED, INFO_WAIT_TIMEOUT, JOB_VALUES, JOB_VECTORS, PREC_FP64,
                       PREC_MIXED, check, lib)

PHASES = ("R1", "R2-4", "S1", "S2", "S3", "S4", "S5", "R5", "REF", "F")

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
    if v == INFO_WAIT_TIMEOUT:
        raise torch.linalg.LinAlgError(f"{where}: a bounded wait between GPU workgroups timed "
                                       f"out; the result is not valid (info={v})")
    if v == INFO_REFINE_FAILED:
        raise torch.linalg.LinAlgError(f"{where}: the mixed-precision refinement met a block of "
                                       f"Y^T B Y that is not positive definite (info={v})")
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


def solve_lowest(A: torch.Tensor, B: torch.Tensor, k: int, check_info=True):
    """All eigenvalues of A y = lambda B y and the eigenvectors of the k smallest.
    Returns (lam [M], Y [M, k]) with Y^T B Y = I_k."""
    A = _square(A, "A")
    B = _square(B, "B")
    M = A.shape[0]
    k = int(k)
    dev = A.device
    lam = torch.empty(M, dtype=torch.float64, device=dev)
    Ycm = torch.empty((max(k, 0), M), dtype=torch.float64, device=dev)  # column-major M x k
    ws = _workspace(lib().gep_workspace_size_lowest(M, k), dev)
    info = _info(dev)
    st = lib().gep_solve_lowest(M, _ptr(A), max(M, 1), _ptr(B), max(M, 1), k, _ptr(lam),
                                _ptr(Ycm), max(M, 1), _ptr(ws), ws.numel(), _ptr(info), _stream())
    check(st, "gep_solve_lowest")
    if check_info:
        _raise_info(info, M, "gep_solve_lowest")
    return lam, Ycm.t()


def solve_cholfree(A: torch.Tensor, B: torch.Tensor, check_info=True):
    """All eigenpairs of A y = lambda B y through the Cholesky-free reducer
    (B W = W D by the SEP solver, C = D^-1/2 W^T A W D^-1/2, Y = W D^-1/2 Z).
    Returns (lam, Y) with Y^T B Y = I."""
    A = _square(A, "A")
    B = _square(B, "B")
    M = A.shape[0]
    dev = A.device
    lam = torch.empty(M, dtype=torch.float64, device=dev)
    Ycm = torch.empty((M, M), dtype=torch.float64, device=dev)  # column-major
    ws = _workspace(lib().gep_workspace_size_cholfree(M), dev)
    info = _info(dev)
    st = lib().gep_solve_cholfree(M, _ptr(A), max(M, 1), _ptr(B), max(M, 1), _ptr(lam), _ptr(Ycm),
                                  max(M, 1), _ptr(ws), ws.numel(), _ptr(info), _stream())
    check(st, "gep_solve_cholfree")
    if check_info:
        v = int(info.item())
        if v > M:
            raise torch.linalg.LinAlgError(f"gep_solve_cholfree: B is not positive definite "
                                           f"({v - M} eigenvalues of B are not positive)")
        _raise_info(info, M, "gep_solve_cholfree")
    return lam, Ycm.t()


def solve_explicit_inverse(A: torch.Tensor, B: torch.Tensor, check_info=True):
    """All eigenpairs of A y = lambda B y through the explicit-inverse (ELPA-style)
    reducer: R = L^-1 formed explicitly, C = (R A) R^T, Y = R^T Z.  Returns (lam, Y)
    with Y^T B Y = I."""
    A = _square(A, "A")
    B = _square(B, "B")
    M = A.shape[0]
    dev = A.device
    lam = torch.empty(M, dtype=torch.float64, device=dev)
    Ycm = torch.empty((M, M), dtype=torch.float64, device=dev)  # column-major
    ws = _workspace(lib().gep_workspace_size_explicit_inverse(M), dev)
    info = _info(dev)
    st = lib().gep_solve_explicit_inverse(M, _ptr(A), max(M, 1), _ptr(B), max(M, 1), _ptr(lam),
                                          _ptr(Ycm), max(M, 1), _ptr(ws), ws.numel(), _ptr(info),
                                          _stream())
    check(st, "gep_solve_explicit_inverse")
    if check_info:
        _raise_info(info, M, "gep_solve_explicit_inverse")
    return lam, Ycm.t()


def solve_jacobi(A: torch.Tensor, B: torch.Tensor, check_info=True):
    """All eigenpairs of A y = lambda B y through the reducer and the parallel block
    Jacobi SEP solver (gep_solve_jacobi).  Returns (lam, Y) with Y^T B Y = I."""
    A = _square(A, "A")
    B = _square(B, "B")
    M = A.shape[0]
    dev = A.device
    lam = torch.empty(M, dtype=torch.float64, device=dev)
    Ycm = torch.empty((M, M), dtype=torch.float64, device=dev)  # column-major
    ws = _workspace(lib().gep_workspace_size_jacobi(M), dev)
    info = _info(dev)
    st = lib().gep_solve_jacobi(M, _ptr(A), max(M, 1), _ptr(B), max(M, 1), _ptr(lam), _ptr(Ycm),
                                max(M, 1), _ptr(ws), ws.numel(), _ptr(info), _stream())
    check(st, "gep_solve_jacobi")
    if check_info:
        _raise_info(info, M, "gep_solve_jacobi")
    return lam, Ycm.t()


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
          lower_only=False, fp32_arith=False):
    """C = alpha A B + beta C on libgep's MFMA GEMM (row-major torch views are
    handled as transposed column-major operands).  fp32_arith: interior tiles in
    FP32 arithmetic (FP64 storage)."""
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
                         _ptr(A), max(k, 1), float(beta), _ptr(C), max(n, 1),
                         1 if fp32_arith else 0, _stream())
    check(st, "gep_dgemm")
    return C


def profile_enable(on: bool = True) -> None:
    lib().gep_profile_enable(1 if on else 0)


def profile_read() -> dict:
    buf = (ctypes.c_double * len(PHASES))()
    n = lib().gep_profile_read(ctypes.cast(buf, ctypes.c_void_p), len(PHASES))
    return {PHASES[i]: buf[i] for i in range(n)}


PROBE_KERNELS = ("dgemm_fast_kernel", "q2_apply", "chase", "panel_qr_coop")


def probe_enable(on: bool = True) -> None:
    """Record HIP events around every launch of the probed kernels (see gep.h)."""
    check(lib().gep_probe_enable(1 if on else 0), "gep_probe_enable")


def probe_read() -> dict:
    """{kernel name: (launches, summed ms, summed algorithmic flops)} since the last
    read; synchronises on the recorded events."""
    out = {}
    for i, name in enumerate(PROBE_KERNELS):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        fl = ctypes.c_double(0.0)
        check(lib().gep_probe_read(i, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl)),
              "gep_probe_read")
        out[name] = (int(n.value), float(ms.value), float(fl.value))
    return out


class BatchedSolver:
    """Solves a fixed list of problems (orders known up front) repeatedly.  Buffers
    and the workspace are allocated once; run() enqueues gep_solve_batched on the
    current stream (so it can be captured in a torch.cuda.CUDAGraph and replayed).
    """

    def __init__(self, sizes, job="vectors", device="cuda:0"):
        self.sizes = [int(m) for m in sizes]
        self.job = _JOBS[job]
        dev = torch.device(device)
        n = len(self.sizes)
        self.A = [torch.zeros((m, m), dtype=torch.float64, device=dev) for m in self.sizes]
        self.B = [torch.zeros((m, m), dtype=torch.float64, device=dev) for m in self.sizes]
        self.lam = [torch.empty(m, dtype=torch.float64, device=dev) for m in self.sizes]
        self.Ycm = ([torch.empty((m, m), dtype=torch.float64, device=dev) for m in self.sizes]
                    if self.job == JOB_VECTORS else None)
        I64A = ctypes.c_int64 * n
        PA = ctypes.c_void_p * n
        self._M = I64A(*self.sizes)
        self._ld = I64A(*[max(m, 1) for m in self.sizes])
        self._A = PA(*[t.data_ptr() for t in self.A])
        self._B = PA(*[t.data_ptr() for t in self.B])
        self._lam = PA(*[t.data_ptr() for t in self.lam])
        self._Y = PA(*[t.data_ptr() for t in self.Ycm]) if self.Ycm is not None else PA()
        self.ws_bytes = int(lib().gep_workspace_size_batched(n, self._M, self.job, PREC_FP64))
        self.ws = _workspace(self.ws_bytes, dev)
        self.info = torch.zeros(n, dtype=torch.int32, device=dev)

    def load(self, As, Bs):
        for dst, src in zip(self.A, As):
            dst.copy_(src)
        for dst, src in zip(self.B, Bs):
            dst.copy_(src)

    def run(self):
        n = len(self.sizes)
        st = lib().gep_solve_batched(n, self._M, self._A, self._ld, self._B, self._ld, self._lam,
                                     self._Y, self._ld, self.job, PREC_FP64, _ptr(self.ws),
                                     self.ws.numel(), _ptr(self.info), _stream())
        check(st, "gep_solve_batched")

    def results(self):
        Ys = [Y.t() for Y in self.Ycm] if self.Ycm is not None else [None] * len(self.sizes)
        return list(zip(self.lam, Ys))


class BatchedGraph:
    """A fixed batch solved by graph replay.  The instances are split largest-first
    (each to the group with the least sum of M^3) into `groups` sub-batches; each
    sub-batch is one BatchedSolver whose gep_solve_batched call is captured in its
    own graph on its own stream, and replay() launches all graphs concurrently.
    (The HIP runtime here replays the parallel branches of a single captured graph
    one node after another, so one graph of the whole batch replays about 2.4x
    slower than the eager call; per-group graphs on separate streams keep the
    groups concurrent.)  Results are identical to one BatchedSolver of the whole
    batch: every instance runs the same kernels either way.  Concurrency between
    streams needs enough hardware queues in the process: HIP's default
    GPU_MAX_HW_QUEUES of 4 folds the streams onto 4 queues (set it, e.g. to 32,
    before HIP initialises).
    """

    def __init__(self, sizes, groups=16, job="vectors", device="cuda:0"):
        self.sizes = [int(m) for m in sizes]
        groups = max(1, min(int(groups), len(self.sizes)))
        order = sorted(range(len(self.sizes)), key=lambda i: -self.sizes[i])
        self.members = [[] for _ in range(groups)]
        load = [0] * groups
        for i in order:
            g = min(range(groups), key=lambda k: load[k])
            self.members[g].append(i)
            load[g] += self.sizes[i] ** 3
        self.members = [m for m in self.members if m]
        self.solvers = [BatchedSolver([self.sizes[i] for i in m], job=job, device=device)
                        for m in self.members]
        self.streams = [torch.cuda.Stream(device=device) for _ in self.members]
        self.graphs = None

    def load(self, As, Bs):
        for m, sv in zip(self.members, self.solvers):
            sv.load([As[i] for i in m], [Bs[i] for i in m])

    def _each(self, fn):
        cur = torch.cuda.current_stream()
        for st, item in zip(self.streams, fn):
            st.wait_stream(cur)
            with torch.cuda.stream(st):
                item()
        for st in self.streams:
            cur.wait_stream(st)

    def run(self):
        """Eager: every group's call on its own stream."""
        self._each([sv.run for sv in self.solvers])

    def capture(self):
        self.run()
        torch.cuda.synchronize()
        self.graphs = []
        for st, sv in zip(self.streams, self.solvers):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(st):
                with torch.cuda.graph(g, stream=st):
                    sv.run()
            self.graphs.append(g)
        torch.cuda.synchronize()

    def replay(self):
        if self.graphs is None:
            raise RuntimeError("BatchedGraph.replay() before capture()")
        self._each([g.replay for g in self.graphs])

    @property
    def info(self):
        out = torch.empty(len(self.sizes), dtype=torch.int32, device=self.solvers[0].info.device)
        for m, sv in zip(self.members, self.solvers):
            out[torch.tensor(m, device=out.device)] = sv.info
        return out

    def results(self):
        out = [None] * len(self.sizes)
        for m, sv in zip(self.members, self.solvers):
            for i, r in zip(m, sv.results()):
                out[i] = r
        return out


def solve_batched(As, Bs, job="vectors", check_info=True):
    """Solve A_i y = lambda B_i y for lists of square float64 CUDA tensors of
    possibly different orders.  Returns a list of (lam, Y)."""
    bs = BatchedSolver([A.shape[0] for A in As], job=job, device=As[0].device)
    bs.load(As, Bs)
    bs.run()
    if check_info:
        info = bs.info.cpu().tolist()
        bad = [i for i, v in enumerate(info) if v != 0]
        if bad:
            raise torch.linalg.LinAlgError(f"gep_solve_batched: instances {bad} failed "
                                           f"(info {[info[i] for i in bad]})")
    return bs.results()


def backward(lam, Y, lam_bar=None, Y_bar=None, eta=0.0, tau_c=0.0):
    """Reverse-mode adjoint of solve(): symmetric (A_bar, B_bar) from the solution
    (lam, Y) and the cotangents lam_bar = dL/dlam, Y_bar = dL/dY (None = zero)."""
    lam = lam.contiguous()
    M = lam.numel()
    dev = lam.device
    Ycm = Y.t().contiguous()  # column-major buffer of Y
    Ybcm = Y_bar.t().contiguous() if Y_bar is not None else None
    lb = lam_bar.contiguous() if lam_bar is not None else None
    Ab = torch.empty((M, M), dtype=torch.float64, device=dev)
    Bb = torch.empty((M, M), dtype=torch.float64, device=dev)
    ws = _workspace(lib().gep_backward_workspace_size(M), dev)
    st = lib().gep_backward(M, _ptr(lam), _ptr(Ycm), max(M, 1), _ptr(lb), _ptr(Ybcm), max(M, 1),
                            float(eta), float(tau_c), _ptr(Ab), max(M, 1), _ptr(Bb), max(M, 1),
                            _ptr(ws), ws.numel(), _stream())
    check(st, "gep_backward")
    return Ab, Bb  # symmetric: row- and column-major agree


class GEPFunction(torch.autograd.Function):
    """(A, B) -> (lam, Y) with the libgep adjoint as backward.  A and B are symmetric
    float64 CUDA tensors; the gradients returned are the symmetric ones (the
    derivative along symmetric perturbations), as torch.linalg.eigh does.
    Degeneracy handling: eta (Lorentzian broadening) and tau_c (coupling cut-off)
    are taken from GEPFunction.eta / GEPFunction.tau_c."""

    eta = 0.0
    tau_c = 0.0

    @staticmethod
    def forward(ctx, A, B):
        lam, Y = solve(A, B)
        ctx.save_for_backward(lam, Y)
        return lam, Y

    @staticmethod
    def backward(ctx, lam_bar, Y_bar):
        lam, Y = ctx.saved_tensors
        Ab, Bb = backward(lam, Y, lam_bar, Y_bar, GEPFunction.eta, GEPFunction.tau_c)
        return Ab, Bb
