"""gep_solve_noalloc (the solve whose workspace is a fixed array in the library's
device image) against gep_solve with a caller-provided workspace, through the C
ABI: two calls in a row, the second on a smaller problem (so it runs over the
first call's leftovers in the shared array), each compared to gep_solve on the
same inputs at the FP64 path's bar (|d lambda| / |A|_1 <= 1e-11, eigenvector
B-angles within clusters), plus an eigenvalues-only and a mixed-precision call,
and the rejection of a problem beyond the array's size."""
import ctypes

import numpy as np
import pytest

import synth
from tests.gpu_util import max_subspace_sine, say, to_gpu, to_np

pytestmark = pytest.mark.gpu

P = ctypes.c_void_p


def _lib():
    from paper_1504_06443_amd import _binding
    return _binding.lib()


def _call(entry, dA, dB, job=1, prec=0):
    import torch
    L = _lib()
    M = dA.shape[0]
    dev = dA.device
    lam = torch.empty(M, dtype=torch.float64, device=dev)
    Y = torch.empty((M, M), dtype=torch.float64, device=dev)  # column-major M x M
    info = torch.full((1,), 777, dtype=torch.int32, device=dev)
    st_ = P(torch.cuda.current_stream().cuda_stream)
    if entry == "noalloc":
        st = L.gep_solve_noalloc(M, P(dA.data_ptr()), M, P(dB.data_ptr()), M, P(lam.data_ptr()),
                                 P(Y.data_ptr()), M, job, prec, P(info.data_ptr()), st_)
    else:
        ws = torch.empty(L.gep_workspace_size(M, job, prec), dtype=torch.uint8, device=dev)
        st = L.gep_solve(M, P(dA.data_ptr()), M, P(dB.data_ptr()), M, P(lam.data_ptr()),
                         P(Y.data_ptr()), M, job, prec, P(ws.data_ptr()), ws.numel(),
                         P(info.data_ptr()), st_)
    torch.cuda.synchronize()
    assert st == 0, (entry, st)
    assert int(info.item()) == 0, (entry, int(info.item()))
    return to_np(lam), to_np(Y).T


def _compare(A, B, got, ref, vectors=True):
    n1 = np.abs(A).sum(axis=0).max()
    err = np.abs(got[0] - ref[0]).max() / n1
    assert err <= 1e-11, err
    if vectors:
        worst = max_subspace_sine(got[1], ref[1], B, ref[0], 1e-8 * n1)
        assert worst <= 1e-11 * n1, worst
    same = bool(np.array_equal(got[0], ref[0])) and (not vectors or np.array_equal(got[1], ref[1]))
    return err, same


@pytest.mark.parametrize("order", [(2048, 700)])
def test_noalloc_two_calls_match_gep_solve(gpu, order):
    for M in order:
        say(f"[noalloc] FP64 eigenpairs M={M}")
        A, B = synth.banded_pair(M, synth.decay_length(M), 8800 + M)
        dA, dB = to_gpu(A), to_gpu(B)
        got = _call("noalloc", dA, dB)
        ref = _call("solve", dA, dB)
        err, same = _compare(A, B, got, ref)
        say(f"  |dlambda|/|A|_1 {err:.1e}, bitwise equal: {same}")


def test_noalloc_values_and_mixed(gpu):
    M = 600
    A, B = synth.banded_pair(M, synth.decay_length(M), 8901)
    dA, dB = to_gpu(A), to_gpu(B)
    say(f"[noalloc] eigenvalues only M={M}")
    _compare(A, B, _call("noalloc", dA, dB, job=0), _call("solve", dA, dB, job=0), vectors=False)
    say(f"[noalloc] mixed precision M={M}")
    got = _call("noalloc", dA, dB, prec=1)
    ref = _call("solve", dA, dB, prec=1)
    n1 = np.abs(A).sum(axis=0).max()
    assert np.abs(got[0] - ref[0]).max() / n1 <= 1e-11
    assert np.abs(got[1].T @ B @ got[1] - np.eye(M)).max() <= 1e-8


def test_noalloc_rejects_problems_beyond_its_array(gpu):
    L = _lib()
    cap = L.gep_noalloc_max_bytes()
    M = 2400
    assert L.gep_workspace_size(M, 1, 0) > cap
    fake = P(0x100000)  # never dereferenced: the size check comes first
    st = L.gep_solve_noalloc(M, fake, M, fake, M, fake, fake, M, 1, 0, fake, None)
    assert st == -2  # GEP_ERR_WORKSPACE
    assert L.gep_workspace_size(2048, 1, 0) <= cap
