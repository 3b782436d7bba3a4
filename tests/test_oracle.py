"""Pins for the CPU oracle: closed forms, brute force, invariants and an
independent library, so that the oracle is checked against something other than
itself before it serves as the reference for the GPU library."""
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth


def toeplitz(M, a, b):
    return synth.toeplitz_tridiag(M, a, b)


def sine_basis(M):
    j = np.arange(1, M + 1)[:, None]
    k = np.arange(1, M + 1)[None, :]
    return np.sqrt(2.0 / (M + 1)) * np.sin(j * k * np.pi / (M + 1))


def match_columns_up_to_sign(Y, X):
    s = np.sign(np.sum(Y * X, axis=0))
    s[s == 0] = 1
    return np.abs(Y - X * s[None, :]).max()


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("M", [1, 2, 3, 17, 64, 131])
def test_toeplitz_identity_closed_form(M):
    """A = tridiag(b, a, b), B = I: lambda_k = a + 2 b cos(k pi / (M+1)),
    y_k(j) = sqrt(2/(M+1)) sin(j k pi / (M+1))."""
    a, b = 0.7, -1.3
    A = toeplitz(M, a, b)
    r = oracle.solve(A, np.eye(M))
    k = np.arange(1, M + 1)
    exact = np.sort(a + 2 * b * np.cos(k * np.pi / (M + 1)))
    assert np.abs(r.lam - exact).max() <= 1e-14 * (abs(a) + 2 * abs(b))
    # eigenvectors: with b < 0 the k-th sine vector belongs to the k-th smallest value
    X = sine_basis(M)
    assert match_columns_up_to_sign(r.Y, X) <= 1e-12


@pytest.mark.parametrize("M", [5, 40, 100])
def test_generalized_toeplitz_pair_closed_form(M):
    """A = tridiag(b, a, b), B = tridiag(d, c, d) with c > 2|d| share the sine
    eigenvectors s_k, so lambda_k = (a + 2b cos t_k)/(c + 2d cos t_k) and
    y_k = s_k / sqrt(c + 2d cos t_k), t_k = k pi/(M+1)."""
    a, b, c, d = -2.0, 0.9, 1.5, 0.4
    A, B = toeplitz(M, a, b), toeplitz(M, c, d)
    r = oracle.solve(A, B)
    t = np.arange(1, M + 1) * np.pi / (M + 1)
    lam = (a + 2 * b * np.cos(t)) / (c + 2 * d * np.cos(t))
    order = np.argsort(lam)
    assert np.abs(r.lam - lam[order]).max() <= 1e-13
    Yx = (sine_basis(M) / np.sqrt(c + 2 * d * np.cos(t))[None, :])[:, order]
    assert match_columns_up_to_sign(r.Y, Yx) <= 1e-11


def test_total_degeneracy_A_equals_alpha_B():
    A0, B = synth.banded_pair(60, 4.0, 11)
    alpha = -3.25
    r = oracle.solve(alpha * B, B)
    assert np.abs(r.lam - alpha).max() <= 1e-13 * abs(alpha) * 4
    Y = r.Y
    assert np.abs(Y.T @ B @ Y - np.eye(60)).max() <= 1e-12


def test_block_diagonal_union_of_spectra():
    M1, M2 = 23, 31
    A = np.zeros((M1 + M2, M1 + M2))
    A[:M1, :M1] = toeplitz(M1, 1.0, 0.5)
    A[M1:, M1:] = toeplitz(M2, -1.0, 2.0)
    r = oracle.solve(A, np.eye(M1 + M2))
    k1 = np.arange(1, M1 + 1)
    k2 = np.arange(1, M2 + 1)
    exact = np.sort(np.concatenate([1.0 + np.cos(k1 * np.pi / (M1 + 1)),
                                    -1.0 + 4.0 * np.cos(k2 * np.pi / (M2 + 1))]))
    assert np.abs(r.lam - exact).max() <= 1e-13


def test_prescribed_spectrum_with_clusters():
    """A = L_B Q diag(mu) Q^T L_B^T with B = L_B L_B^T has eigenvalues mu exactly,
    including prescribed multiplicities."""
    M = 80
    rng = np.random.default_rng(3)
    _, B = synth.banded_pair(M, 5.0, 12)
    LB = np.linalg.cholesky(B)
    Q, _ = np.linalg.qr(rng.standard_normal((M, M)))
    mu = np.sort(np.concatenate([rng.uniform(-5, 5, M - 10), np.full(6, 1.25), np.full(4, -2.5)]))
    A = LB @ Q @ np.diag(mu) @ Q.T @ LB.T
    A = 0.5 * (A + A.T)
    r = oracle.solve(A, B)
    assert np.abs(r.lam - mu).max() <= 1e-13 * np.abs(mu).max() * 10
    Y = r.Y
    assert np.abs(Y.T @ B @ Y - np.eye(M)).max() <= 1e-12
    assert np.abs(A @ Y - B @ Y * r.lam[None, :]).max() <= 1e-12 * r.norm1


# ---------------------------------------------------------------- brute force

def _frac_det(Mx):
    n = len(Mx)
    a = [row[:] for row in Mx]
    det = Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if a[r][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            a[c], a[p] = a[p], a[c]
            det = -det
        det *= a[c][c]
        for r in range(c + 1, n):
            f = a[r][c] / a[c][c]
            if f:
                for k in range(c, n):
                    a[r][k] -= f * a[c][k]
    return det


def brute_force_eigvals(A, B, dps=50):
    """Roots of det(A - x B), whose coefficients are found exactly in rational
    arithmetic by evaluating the determinant at M+1 integer points and solving the
    Vandermonde system, then located with mpmath at `dps` digits."""
    M = A.shape[0]
    Af = [[Fraction(float(v)) for v in row] for row in A]
    Bf = [[Fraction(float(v)) for v in row] for row in B]
    xs = [Fraction(x) for x in range(M + 1)]
    vals = [_frac_det([[Af[i][j] - x * Bf[i][j] for j in range(M)] for i in range(M)]) for x in xs]
    # Vandermonde solve (exact): coefficients c_0..c_M of sum c_k x^k
    V = [[x ** k for k in range(M + 1)] + [v] for x, v in zip(xs, vals)]
    n = M + 1
    for c in range(n):
        p = next(r for r in range(c, n) if V[r][c] != 0)
        V[c], V[p] = V[p], V[c]
        for r in range(n):
            if r != c and V[r][c] != 0:
                f = V[r][c] / V[c][c]
                for k in range(c, n + 1):
                    V[r][k] -= f * V[c][k]
    coef = [V[k][n] / V[k][k] for k in range(n)]
    with mpmath.workdps(dps):
        mc = [mpmath.mpf(c.numerator) / c.denominator for c in reversed(coef)]
        roots = mpmath.polyroots(mc, maxsteps=400, extraprec=400)
        re = sorted(float(mpmath.re(z)) for z in roots)
        assert max(abs(float(mpmath.im(z))) for z in roots) < 1e-20
    return np.array(re)


@pytest.mark.parametrize("M,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (8, 4), (8, 5)])
def test_brute_force_small(M, seed):
    A, B = synth.banded_pair(M, 2.0, 100 + seed)
    exact = brute_force_eigvals(A, B)
    r = oracle.solve(A, B)
    assert np.abs(r.lam - exact).max() <= 1e-14 * max(1.0, r.norm1)
    Y = r.Y
    assert np.abs(Y.T @ B @ Y - np.eye(M)).max() <= 1e-14
    assert np.abs(A @ Y - B @ Y * r.lam[None, :]).max() <= 1e-14 * max(1.0, r.norm1)


# ---------------------------------------------------------------- steps

def test_cholesky_unique_factor_and_failure():
    _, B = synth.banded_pair(70, 5.0, 13)
    L, info = oracle.cholesky(B)
    assert info == 0
    assert np.allclose(np.triu(L, 1), 0.0)
    assert np.all(np.diag(L) > 0)
    assert np.abs(L @ L.T - B).max() <= 1e-15 * 8
    # the factor with positive diagonal is unique: an independent library agrees
    assert np.abs(L - np.linalg.cholesky(B)).max() <= 1e-14
    # a negative leading minor of order k is reported as k
    Bbad = B.copy()
    Bbad[9, 9] = -1.0
    _, info = oracle.cholesky(Bbad)
    assert info == 10
    r = oracle.solve(np.eye(70), Bbad)
    assert r.info == 70 + 10


def test_reduce_and_back_transform_identities():
    A, B = synth.banded_pair(90, 6.0, 14)
    L, _ = oracle.cholesky(B)
    C = oracle.reduce(A, L)
    assert np.abs(C - C.T).max() == 0.0
    assert np.abs(L @ C @ L.T - A).max() <= 1e-13
    Z = np.random.default_rng(0).standard_normal((90, 7))
    Y = oracle.back_transform(L, Z)
    assert np.abs(L.T @ Y - Z).max() <= 1e-13


def test_tridiagonalization_similarity():
    A, B = synth.banded_pair(75, 6.0, 15)
    L, _ = oracle.cholesky(B)
    C = oracle.reduce(A, L)
    d, e, R, beta = oracle.tridiagonalize(C)
    T = np.diag(d) + np.diag(e, -1) + np.diag(e, 1)
    Q = oracle.form_q(R, beta)
    assert np.abs(Q.T @ Q - np.eye(75)).max() <= 1e-14
    assert np.abs(Q @ T @ Q.T - C).max() <= 1e-13 * np.abs(C).max() * 10
    # Sturm counts agree with an independent symmetric eigen-solver on C
    w = np.linalg.eigvalsh(C)
    for x in np.linspace(w[0] - 1, w[-1] + 1, 23):
        if np.min(np.abs(w - x)) > 1e-9:
            assert oracle.sturm_count(d, e, x) == int(np.sum(w < x))


@pytest.mark.parametrize("M", [2, 9, 50, 257])
def test_clement_matrix(M):
    """Clement/Kac matrix: zero diagonal, off-diagonals sqrt(i (M - i)); its
    eigenvalues are -(M-1), -(M-3), ..., (M-1)."""
    i = np.arange(1, M)
    d = np.zeros(M)
    e = np.sqrt(i * (M - i)).astype(np.float64)
    exact = np.arange(-(M - 1), M, 2, dtype=np.float64)
    w = oracle.tridiag_eigvals(d, e)
    assert np.abs(w - exact).max() <= 1e-13 * M
    wq, Z, info = oracle.tql(d, e, np.eye(M))
    assert info == 0
    assert np.abs(np.sort(wq) - exact).max() <= 1e-12 * M
    T = np.diag(d) + np.diag(e, -1) + np.diag(e, 1)
    assert np.abs(T @ Z - Z * wq[None, :]).max() <= 1e-12 * M
    assert np.abs(Z.T @ Z - np.eye(M)).max() <= 1e-13 * M


def test_invariants_trace_and_frobenius():
    A, B = synth.banded_pair(128, 8.0, 16)
    r = oracle.solve(A, B, keep=True)
    C = r.C
    assert abs(r.lam.sum() - np.trace(C)) <= 1e-12 * np.abs(C).sum()
    assert abs((r.lam ** 2).sum() - (C ** 2).sum()) <= 1e-12 * (C ** 2).sum()


def test_library_cross_check_c1_size():
    """At the 512 size, the oracle agrees with LAPACK's generalized driver."""
    A, B = synth.workload("m512")
    r = oracle.solve(A, B)
    w, V = sla.eigh(A, B)
    assert np.abs(r.lam - w).max() <= 1e-13 * r.norm1
    Y = r.Y
    assert np.abs(Y.T @ B @ Y - np.eye(512)).max() <= 1e-12
    res = np.abs(A @ Y - B @ Y * r.lam[None, :]).sum(axis=0).max()
    assert res <= 1e-12 * r.norm1 * np.abs(Y).sum(axis=0).max()


def test_qr_and_bisection_agree():
    A, B = synth.banded_pair(200, 10.0, 17)
    r = oracle.solve(A, B, keep=True)
    wq, Z, info = oracle.tql(r.d, r.e, np.eye(200))
    assert np.abs(np.sort(wq) - r.lam).max() <= 1e-13 * r.norm1


def test_sign_convention():
    A, B = synth.banded_pair(40, 3.0, 18)
    Y = oracle.solve(A, B).Y
    idx = np.argmax(np.abs(Y), axis=0)
    assert np.all(Y[idx, np.arange(40)] > 0)


def test_empty_and_scalar():
    r = oracle.solve(np.zeros((0, 0)), np.zeros((0, 0)))
    assert r.lam.size == 0 and r.info == 0
    r = oracle.solve(np.array([[3.0]]), np.array([[4.0]]))
    assert abs(r.lam[0] - 0.75) <= 4e-16 and abs(r.Y[0, 0] - 0.5) < 1e-16


# ---------------------------------------------------------------- adjoint

def _loss(A, B, G, nocc):
    r = oracle.solve(A, B)
    Yo = r.Y[:, :nocc]
    return r.lam[:nocc].sum() + np.sum(G * (Yo @ Yo.T))


def _grad_of_loss(A, B, G, nocc, tau_c=0.0):
    r = oracle.solve(A, B)
    M = A.shape[0]
    lam_bar = np.zeros(M)
    lam_bar[:nocc] = 1.0
    Y_bar = np.zeros((M, M))
    Y_bar[:, :nocc] = 2.0 * G @ r.Y[:, :nocc]
    return oracle.gradient(r.lam, r.Y, lam_bar, Y_bar, 0.0, tau_c)


@pytest.mark.parametrize("M", [12, 40])
def test_gradient_vs_central_differences(M):
    A, B = synth.banded_pair(M, 3.0, 19)
    G = synth.symmetric_normal(M, 20, 1.0 / np.sqrt(M))
    nocc = M // 2
    Ab, Bb = _grad_of_loss(A, B, G, nocc)
    h = 1e-6
    for d in range(6):
        E = synth.unit_direction(M, 30 + d)
        dA = E if d % 3 != 1 else 0 * E
        dB = 0.1 * E if d % 3 != 0 else 0 * E
        fd = (_loss(A + h * dA, B + h * dB, G, nocc) - _loss(A - h * dA, B - h * dB, G, nocc)) / (2 * h)
        an = np.sum(Ab * dA) + np.sum(Bb * dB)
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an))


def test_gradient_eigenvalue_sum_closed_form():
    """d(sum_{k<=n} lambda_k)/dA = Y_o Y_o^T and /dB = -Y_o Lambda_o Y_o^T."""
    A, B = synth.banded_pair(30, 3.0, 21)
    r = oracle.solve(A, B)
    lb = np.zeros(30)
    lb[:15] = 1.0
    Ab, Bb = oracle.gradient(r.lam, r.Y, lb, None)
    Yo = r.Y[:, :15]
    assert np.abs(Ab - Yo @ Yo.T).max() <= 1e-13
    assert np.abs(Bb + Yo @ np.diag(r.lam[:15]) @ Yo.T).max() <= 1e-12


def test_gradient_with_exact_degeneracy_inside_occupied_set():
    """A loss invariant under rotations of a degenerate occupied eigenspace still
    has a well-defined gradient; zeroing F inside the cluster gives it."""
    M = 24
    rng = np.random.default_rng(5)
    _, B = synth.banded_pair(M, 3.0, 22)
    LB = np.linalg.cholesky(B)
    Q, _ = np.linalg.qr(rng.standard_normal((M, M)))
    mu = np.sort(rng.uniform(-4, 4, M))
    mu[3:6] = mu[3]  # triple eigenvalue in the occupied half
    A = LB @ Q @ np.diag(mu) @ Q.T @ LB.T
    A = 0.5 * (A + A.T)
    G = synth.symmetric_normal(M, 23, 1.0 / np.sqrt(M))
    nocc = M // 2
    Ab, Bb = _grad_of_loss(A, B, G, nocc, tau_c=1e-8)
    h = 1e-6
    for d in range(4):
        E = synth.unit_direction(M, 40 + d)
        dA, dB = (E, 0 * E) if d % 2 == 0 else (0 * E, 0.1 * E)
        fd = (_loss(A + h * dA, B + h * dB, G, nocc) - _loss(A - h * dA, B - h * dB, G, nocc)) / (2 * h)
        an = np.sum(Ab * dA) + np.sum(Bb * dB)
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an))


# ---------------------------------------------------------------- generator

def test_generator_deterministic_and_spd():
    A1, B1 = synth.banded_pair(700, 8.0, 1)
    A2, B2 = synth.banded_pair(700, 8.0, 1)
    assert np.array_equal(A1, A2) and np.array_equal(B1, B2)
    assert np.array_equal(A1, A1.T) and np.array_equal(B1, B1.T)
    off = np.abs(B1 - np.diag(np.diag(B1))).sum(axis=1)
    assert abs(off.max() - 0.5) < 1e-12
    assert np.all(np.diag(B1) == 1.0)
    assert np.all((np.diag(A1) >= -10) & (np.diag(A1) <= 0))
    w = np.linalg.eigvalsh(B1)
    assert w.min() >= 0.5 - 1e-12 and w.max() <= 1.5 + 1e-12


def test_batch_sizes_in_range():
    s = synth.batch_sizes()
    assert len(s) == 256 and min(s) >= 64 and max(s) <= 2048
    assert s == synth.batch_sizes()


def test_inertia_count_matches_eigenvalues():
    """Sylvester count at sigma between eigenvalues, and at an eigenvalue of a
    known degenerate pencil, against the oracle's own eigenvalues."""
    A, B = synth.banded_pair(300, 5.0, 91)
    lam = oracle.solve(A, B, vectors=False).lam
    for k in (0, 1, 17, 150, 299):
        lo = lam[k - 1] if k > 0 else lam[0] - 1.0
        sigma = 0.5 * (lo + lam[k]) if k > 0 else lam[0] - 1.0
        assert oracle.inertia_count(A, B, sigma) == k
    assert oracle.inertia_count(A, B, lam[-1] + 1.0) == 300
    # A = alpha B: every eigenvalue equals alpha
    assert oracle.inertia_count(-2.0 * B, B, -2.0 - 1e-9) == 0
    assert oracle.inertia_count(-2.0 * B, B, -2.0 + 1e-9) == 300
    # 2 x 2 pivots: a pencil whose A has a zero diagonal forces them
    J = np.kron(np.eye(40), np.array([[0.0, 1.0], [1.0, 0.0]]))
    assert oracle.inertia_count(J, np.eye(80), 0.0) == 40
    assert oracle.inertia_count(J, np.eye(80), -1.5) == 0
    assert oracle.inertia_count(J, np.eye(80), 1.5) == 80


def test_inertia_count_pivot_cases_against_numpy():
    """The oracle's own indefinite factorisation against LAPACK's symmetric
    eigenvalue count (numpy.linalg.eigvalsh) on matrices that exercise each pivot
    choice: dominant diagonal (1 x 1 in place), zero or tiny diagonal with large
    off-diagonal (2 x 2 blocks), a large entry far below the diagonal (row and
    column interchanges), a 2 x 2 block with positive determinant and negative
    trace, and an exactly singular pivot (ValueError)."""
    rng = np.random.default_rng(4242)
    cases = []
    for n in (3, 8, 33, 120, 301):
        X = rng.standard_normal((n, n))
        cases.append(0.5 * (X + X.T))                      # generic indefinite
        Z = 0.5 * (X + X.T)
        np.fill_diagonal(Z, 0.0)
        cases.append(Z)                                     # zero diagonal
        D = Z.copy()
        np.fill_diagonal(D, 1e-8 * rng.standard_normal(n))
        D[n - 1, 0] = D[0, n - 1] = 50.0                    # far pivot row
        cases.append(D)
        T = np.diag(rng.uniform(1, 2, n) * rng.choice([-1.0, 1.0], n))
        cases.append(T + 1e-3 * Z)                          # 1 x 1 pivots
    # 2 x 2 blocks with det > 0, trace < 0: [[-1, 0.5], [0.5, -1]] inside zero diagonal
    K = np.kron(np.eye(20), np.array([[-0.01, 3.0], [3.0, -0.02]]))
    cases.append(K)
    for S in cases:
        n = S.shape[0]
        w = np.linalg.eigvalsh(S)
        gap = np.min(np.abs(w))
        assert gap > 1e-10, "case must be nonsingular"
        assert oracle.inertia_count(S, np.eye(n), 0.0) == int((w < 0).sum())
        # a shift between two eigenvalues, B a general SPD matrix
        _, Bs = synth.banded_pair(n, 2.0, 7 + n)
        lam = np.linalg.eigvalsh(np.linalg.solve(np.linalg.cholesky(Bs), np.linalg.solve(
            np.linalg.cholesky(Bs), S).T))
        k = n // 2
        if k > 0 and lam[k] - lam[k - 1] > 1e-8:
            assert oracle.inertia_count(S, Bs, 0.5 * (lam[k - 1] + lam[k])) == k
    with pytest.raises(ValueError):
        oracle.inertia_count(np.zeros((4, 4)), np.eye(4), 0.0)


@pytest.mark.parametrize("name", ["m8192", "m32768"])
def test_stored_eigenvalues_agree_with_stored_inertia(name):
    """The two stored references of a workload come from independent routes of the
    oracle (bisection on the tridiagonal matrix for the eigenvalues; a symmetric
    indefinite factorisation of A - sigma B for the counts): the number of stored
    eigenvalues below each shift must equal the stored count."""
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    pe, pc = os.path.join(here, f"{name}_eigenvalues.npy"), os.path.join(here, f"{name}_inertia.json")
    if not (os.path.exists(pe) and os.path.exists(pc)):
        pytest.skip(f"{name}: stored eigenvalues or counts not present")
    lam = np.load(pe)
    for s, c in json.load(open(pc))["counts_below_sigma"].items():
        assert int(np.count_nonzero(lam < float(s))) == c, s
