"""GPU checks of the device-side failure reports: the bounded waits of the band
reduction's grid barrier and of the bulge chase, and the tridiagonal solver's
non-convergence, each forced from the host (the kernels' own waits give up at
their first unsatisfied poll, or the leaf solver's iteration cap is zero), so
that every kernel still exits normally.  The solve must then return status OK
and report the failure in the device info word; with the switch off again the
next solve is correct."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import say, to_gpu, to_np

pytestmark = pytest.mark.gpu

WAIT_TIMEOUT = -1


def _lib():
    from paper_1504_06443_amd import _binding
    return _binding.lib()


def _raw_solve(A, B, job=1, prec=0, entry="gep_solve"):
    """One call through the C ABI; returns (status, info, lam, Y)."""
    import torch
    L = _lib()
    M = A.shape[0]
    dev = A.device
    lam = torch.empty(M, dtype=torch.float64, device=dev)
    Y = torch.empty((M, M), dtype=torch.float64, device=dev)
    info = torch.full((1,), 12345, dtype=torch.int32, device=dev)
    st_ = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = ctypes.c_void_p
    if entry == "gep_solve":
        ws = torch.empty(L.gep_workspace_size(M, job, prec), dtype=torch.uint8, device=dev)
        st = L.gep_solve(M, P(A.data_ptr()), M, P(B.data_ptr()), M, P(lam.data_ptr()),
                         P(Y.data_ptr()), M, job, prec, P(ws.data_ptr()), ws.numel(),
                         P(info.data_ptr()), st_)
    elif entry == "gep_solve_cholfree":
        ws = torch.empty(L.gep_workspace_size_cholfree(M), dtype=torch.uint8, device=dev)
        st = L.gep_solve_cholfree(M, P(A.data_ptr()), M, P(B.data_ptr()), M, P(lam.data_ptr()),
                                  P(Y.data_ptr()), M, P(ws.data_ptr()), ws.numel(),
                                  P(info.data_ptr()), st_)
    else:
        raise ValueError(entry)
    torch.cuda.synchronize()
    return st, int(info.item()), lam, Y


@pytest.fixture
def inputs(gpu):
    M = 600
    A, B = synth.banded_pair(M, 8.0, 9601)
    return A, B, to_gpu(A), to_gpu(B)


def _recovered(A, B, dA, dB):
    """With the switches off, the next solve succeeds and matches the oracle."""
    st, info, lam, _ = _raw_solve(dA, dB)
    assert st == 0 and info == 0, (st, info)
    ref = oracle.solve(A, B, vectors=False)
    err = np.abs(to_np(lam) - ref.lam).max() / ref.norm1
    assert err <= 1e-11, err


@pytest.mark.parametrize("job,prec,entry", [(1, 0, "gep_solve"), (0, 0, "gep_solve"),
                                            (1, 1, "gep_solve"), (1, 0, "gep_solve_cholfree")])
def test_forced_wait_timeout_reaches_info(inputs, job, prec, entry):
    A, B, dA, dB = inputs
    say(f"[failures] forced wait timeout: {entry} job={job} prec={prec} M={A.shape[0]}")
    L = _lib()
    assert L.gep_debug_force_wait_timeout(1) == 0
    try:
        st, info, _, _ = _raw_solve(dA, dB, job, prec, entry)
    finally:
        L.gep_debug_force_wait_timeout(0)
    assert st == 0
    assert info == WAIT_TIMEOUT, info
    _recovered(A, B, dA, dB)


def test_forced_wait_timeout_raises_in_python(inputs):
    import torch
    A, B, dA, dB = inputs
    say("[failures] forced wait timeout through the Python API")
    import paper_1504_06443_amd as gep
    L = _lib()
    L.gep_debug_force_wait_timeout(1)
    try:
        with pytest.raises(torch.linalg.LinAlgError, match="timed out"):
            gep.solve(dA, dB)
    finally:
        L.gep_debug_force_wait_timeout(0)
    _recovered(A, B, dA, dB)


def test_forced_eig_failure_reaches_info(inputs):
    A, B, dA, dB = inputs
    M = A.shape[0]
    say(f"[failures] forced tridiagonal non-convergence M={M}")
    L = _lib()
    assert L.gep_debug_force_eig_failure(1) == 0
    try:
        st_v, info_v, _, _ = _raw_solve(dA, dB, job=1)
        st_e, info_e, _, _ = _raw_solve(dA, dB, job=0)  # bisection: no QL, unaffected
    finally:
        L.gep_debug_force_eig_failure(0)
    assert st_v == 0 and 1 <= info_v <= M, info_v  # a leaf's first index + 1
    assert st_e == 0 and info_e == 0, info_e
    _recovered(A, B, dA, dB)
