"""CPU-side checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments on the host before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gep.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gep_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1504_06443_amd import _binding
    return _binding.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("gep_solve", "gep_workspace_size", "gep_status_string", "gep_reduce",
              "gep_tridiag_eig", "gep_band_reduce", "gep_tridiagonalize"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    assert lib.gep_status_string(0) == b"ok"
    assert lib.gep_status_string(-1) == b"invalid argument"
    assert lib.gep_status_string(-2) == b"workspace too small"


def test_workspace_sizes_grow(lib):
    s1 = lib.gep_workspace_size(100, 1, 0)
    s2 = lib.gep_workspace_size(1000, 1, 0)
    assert 0 < s1 < s2
    assert lib.gep_workspace_size(1000, 0, 0) < s2
    assert lib.gep_workspace_size(0, 1, 0) > 0


P = ctypes.c_void_p
FAKE = P(0x100000)  # never dereferenced: validation fails first


def _solve(lib, M, lda=None, A=FAKE, B=FAKE, lam=FAKE, Y=FAKE, job=1, prec=0, ws=P(0x200000),
           wsb=None, info=FAKE):
    lda = M if lda is None else lda
    wsb = lib.gep_workspace_size(max(M, 0), job, prec) if wsb is None else wsb
    return lib.gep_solve(M, A, lda, B, max(M, 1), lam, Y, max(M, 1), job, prec, ws, wsb, info, None)


@pytest.mark.parametrize("kwargs,arg", [
    (dict(M=-1), 1),
    (dict(M=10, A=P(0)), 2),
    (dict(M=10, lda=9), 3),
    (dict(M=10, B=P(0)), 4),
    (dict(M=10, lam=P(0)), 6),
    (dict(M=10, Y=P(0)), 7),
    (dict(M=10, job=5), 9),
    (dict(M=10, prec=7), 10),
    (dict(M=10, job=0, prec=1), 10),  # mixed precision refines eigenvectors: vectors only
    (dict(M=10, ws=P(0x200010)), 11),
    (dict(M=10, info=P(0)), 13),
])
def test_solve_rejects_bad_arguments(lib, kwargs, arg):
    assert _solve(lib, **kwargs) == -1
    assert lib.gep_last_bad_arg() == arg


def test_solve_rejects_small_workspace(lib):
    M = 50
    need = lib.gep_workspace_size(M, 1, 0)
    assert _solve(lib, M, wsb=need - 1) == -2


def test_values_job_allows_null_Y(lib):
    # argument checks pass; the call then fails only at the workspace check
    M = 50
    need = lib.gep_workspace_size(M, 0, 0)
    assert _solve(lib, M, Y=P(0), job=0, wsb=need - 1) == -2


def test_phase_entry_points_validate(lib):
    assert lib.gep_reduce(-1, FAKE, 1, FAKE, 1, FAKE, 1, FAKE, 1, FAKE, 10, FAKE, None) == -1
    assert lib.gep_last_bad_arg() == 1
    assert lib.gep_tridiag_eig(5, FAKE, FAKE, FAKE, FAKE, 4, 1, FAKE, 1 << 30, FAKE, None) == -1
    assert lib.gep_last_bad_arg() == 6
    assert lib.gep_band_reduce(5, FAKE, 5, 65, FAKE, 70, FAKE, 1 << 30, None) == -1
    assert lib.gep_last_bad_arg() == 4


def test_mixed_workspace_is_larger(lib):
    assert lib.gep_workspace_size(1000, 1, 1) > lib.gep_workspace_size(1000, 1, 0)


def test_dgemm_rejects_bad_arguments(lib):
    def call(ta=0, tb=0, uplo=0, m=4, n=4, k=4, lda=4, ldb=4, ldc=4, arith=0):
        return lib.gep_dgemm(ta, tb, uplo, m, n, k, 1.0, FAKE, lda, FAKE, ldb, 0.0, FAKE, ldc,
                             arith, None)
    for kw, idx in [(dict(ta=2), 1), (dict(tb=-1), 2), (dict(uplo=1, n=5, ldb=4), 3),
                    (dict(m=-1), 4), (dict(lda=3), 9), (dict(ldc=3), 14), (dict(arith=2), 15)]:
        assert call(**kw) == -1, kw
        assert lib.gep_last_bad_arg() == idx, kw


def test_probe_names_and_bad_index(lib):
    assert lib.gep_probe_name(0) == b"dgemm_fast_kernel"
    assert lib.gep_probe_name(1) == b"q2_apply"
    assert lib.gep_probe_name(4) is None
    assert lib.gep_probe_read(4, None, None, None) == -1
    assert lib.gep_last_bad_arg() == 1


def _lowest(lib, M, k, lda=None, A=FAKE, B=FAKE, lam=FAKE, Y=FAKE, ldy=None, ws=P(0x200000),
            wsb=None, info=FAKE):
    lda = M if lda is None else lda
    ldy = max(M, 1) if ldy is None else ldy
    wsb = lib.gep_workspace_size_lowest(max(M, 0), k) if wsb is None else wsb
    return lib.gep_solve_lowest(M, A, lda, B, max(M, 1), k, lam, Y, ldy, ws, wsb, info, None)


@pytest.mark.parametrize("kwargs,arg", [
    (dict(M=-1, k=0), 1),
    (dict(M=10, k=3, A=P(0)), 2),
    (dict(M=10, k=3, lda=9), 3),
    (dict(M=10, k=3, B=P(0)), 4),
    (dict(M=10, k=-1), 6),
    (dict(M=10, k=11), 6),
    (dict(M=10, k=3, lam=P(0)), 7),
    (dict(M=10, k=3, Y=P(0)), 8),
    (dict(M=10, k=3, ldy=9), 9),
    (dict(M=10, k=3, ws=P(0x200010)), 10),
    (dict(M=10, k=3, info=P(0)), 12),
])
def test_solve_lowest_rejects_bad_arguments(lib, kwargs, arg):
    assert _lowest(lib, **kwargs) == -1
    assert lib.gep_last_bad_arg() == arg


def test_solve_lowest_workspace(lib):
    M = 300
    # k < M holds the tridiagonal solver's M x M eigenvectors on top of gep_solve's needs
    assert lib.gep_workspace_size_lowest(M, M) == lib.gep_workspace_size(M, 1, 0)
    assert lib.gep_workspace_size_lowest(M, 10) >= lib.gep_workspace_size(M, 1, 0) + 8 * M * M
    # k = 0 needs no Y; the call then fails only at the workspace check
    need = lib.gep_workspace_size_lowest(M, 0)
    assert _lowest(lib, M, 0, Y=P(0), wsb=need - 1) == -2



def _cholfree(lib, M, lda=None, A=FAKE, B=FAKE, lam=FAKE, Y=FAKE, ldy=None, ws=P(0x200000),
              wsb=None, info=FAKE):
    lda = M if lda is None else lda
    ldy = max(M, 1) if ldy is None else ldy
    wsb = lib.gep_workspace_size_cholfree(max(M, 0)) if wsb is None else wsb
    return lib.gep_solve_cholfree(M, A, lda, B, max(M, 1), lam, Y, ldy, ws, wsb, info, None)


@pytest.mark.parametrize("kwargs,arg", [
    (dict(M=-1), 1),
    (dict(M=10, A=P(0)), 2),
    (dict(M=10, lda=9), 3),
    (dict(M=10, B=P(0)), 4),
    (dict(M=10, lam=P(0)), 6),
    (dict(M=10, Y=P(0)), 7),
    (dict(M=10, ldy=9), 8),
    (dict(M=10, ws=P(0x200010)), 9),
    (dict(M=10, ws=P(0)), 9),
    (dict(M=10, info=P(0)), 11),
])
def test_solve_cholfree_rejects_bad_arguments(lib, kwargs, arg):
    assert _cholfree(lib, **kwargs) == -1
    assert lib.gep_last_bad_arg() == arg


def test_solve_cholfree_workspace(lib):
    M = 300
    # one M x M buffer (W) and M doubles (D) on top of gep_solve's needs
    base = lib.gep_workspace_size(M, 1, 0)
    assert lib.gep_workspace_size_cholfree(M) >= base + 8 * M * M + 8 * M
    assert lib.gep_workspace_size_cholfree(0) == 256
    need = lib.gep_workspace_size_cholfree(M)
    assert _cholfree(lib, M, wsb=need - 1) == -2


def _explicit(lib, M, lda=None, A=FAKE, B=FAKE, lam=FAKE, Y=FAKE, ldy=None, ws=P(0x200000),
              wsb=None, info=FAKE):
    lda = M if lda is None else lda
    ldy = max(M, 1) if ldy is None else ldy
    wsb = lib.gep_workspace_size_explicit_inverse(max(M, 0)) if wsb is None else wsb
    return lib.gep_solve_explicit_inverse(M, A, lda, B, max(M, 1), lam, Y, ldy, ws, wsb, info,
                                          None)


@pytest.mark.parametrize("kwargs,arg", [
    (dict(M=-1), 1),
    (dict(M=10, A=P(0)), 2),
    (dict(M=10, lda=9), 3),
    (dict(M=10, B=P(0)), 4),
    (dict(M=10, lam=P(0)), 6),
    (dict(M=10, Y=P(0)), 7),
    (dict(M=10, ldy=9), 8),
    (dict(M=10, ws=P(0x200010)), 9),
    (dict(M=10, info=P(0)), 11),
])
def test_solve_explicit_inverse_rejects_bad_arguments(lib, kwargs, arg):
    assert _explicit(lib, **kwargs) == -1
    assert lib.gep_last_bad_arg() == arg


def test_solve_explicit_inverse_workspace(lib):
    M = 300
    # one M x M buffer (R = L^-1) on top of gep_solve's needs
    assert lib.gep_workspace_size_explicit_inverse(M) >= lib.gep_workspace_size(M, 1, 0) + 8 * M * M
    assert lib.gep_workspace_size_explicit_inverse(0) == 256
    need = lib.gep_workspace_size_explicit_inverse(M)
    assert _explicit(lib, M, wsb=need - 1) == -2


def test_tuning_table_api(lib, tmp_path):
    """The tuning table's host logic: built-in rules, overrides (latest covering
    override wins), range and value checks, loading a file and rejecting a
    malformed one (the previous table stays), clearing."""
    get = lambda k, M: lib.gep_tune_get(k.encode(), M)
    lib.gep_tune_clear()
    assert [get("band_width", M) for M in (100, 256, 2047, 2048)] == [16, 32, 32, 64]
    assert get("dc_leaf", 1000) == 64 and get("symm_split_rows", 10) == 2048
    # the ticketed chase is the built-in S2 kernel at every order; the data-stationary
    # one only runs when selected
    assert [get("chase_stationary", M) for M in (3, 600, 8192, 32768)] == [0, 0, 0, 0]
    assert get("no_such_parameter", 10) == -1
    assert lib.gep_tune_set(b"band_width", 100, 200, 24) == 0
    assert lib.gep_tune_set(b"band_width", 150, 160, 48) == 0
    assert (get("band_width", 99), get("band_width", 100), get("band_width", 155)) == (16, 24, 48)
    assert lib.gep_tune_set(b"band_width", 0, 10, 65) == -1      # value out of range
    assert lib.gep_tune_set(b"band_width", 10, 9, 16) == -1      # empty range
    assert lib.gep_tune_set(b"bogus", 0, 10, 16) == -1
    assert lib.gep_tune_set(None, 0, 10, 16) == -1
    lib.gep_tune_reset_overrides()
    assert get("band_width", 155) == 16
    good = tmp_path / "t.json"
    good.write_text('{"device": "x", "parameters": {"band_width": [{"m_lo": 64, "m_hi": 127, '
                    '"value": 24, "ms": 1.5}], "dc_leaf": [{"m_lo": 0, "m_hi": 9999, "value": 32}],'
                    ' "future_parameter": [{"m_lo": 0, "m_hi": 1, "value": 1}]}, "timings": []}')
    assert lib.gep_tune_load(str(good).encode()) == 2
    assert (get("band_width", 100), get("band_width", 300), get("dc_leaf", 5000)) == (24, 32, 32)
    bad = tmp_path / "bad.json"
    for text in ('{"parameters": {"band_width": [{"m_lo": 1, "m_hi": 2, "value": 99}]}}',
                 '{"parameters": {"band_width": [{"m_lo": 1, "value": 16}]}}',
                 '{"parameters": {"band_width": [{"m_lo": 1.5, "m_hi": 2, "value": 16}]}}',
                 '{"parameters": ', '[1, 2]'):
        bad.write_text(text)
        assert lib.gep_tune_load(str(bad).encode()) == -1, text
        assert get("band_width", 100) == 24  # previous table kept
    assert lib.gep_tune_load(str(tmp_path / "missing.json").encode()) == -1
    lib.gep_tune_clear()
    assert get("band_width", 100) == 16
    lib.gep_tune_load(None)  # back to the default location (the committed table, if any)


def test_jacobi_entry_rejects_bad_arguments(lib):
    P = ctypes.c_void_p
    f = P(0x100000)
    w = P(0x200000)
    need = lib.gep_workspace_size_jacobi(50)
    assert need > lib.gep_workspace_size_jacobi(10) > 0
    assert lib.gep_solve_jacobi(-1, f, 1, f, 1, f, f, 1, w, need, f, None) == -1
    assert lib.gep_last_bad_arg() == 1
    assert lib.gep_solve_jacobi(50, f, 49, f, 50, f, f, 50, w, need, f, None) == -1
    assert lib.gep_last_bad_arg() == 3
    assert lib.gep_solve_jacobi(50, f, 50, f, 50, f, f, 50, w, need, None, None) == -1
    assert lib.gep_last_bad_arg() == 11
    assert lib.gep_solve_jacobi(50, f, 50, f, 50, f, f, 50, w, need - 1, f, None) == -2
