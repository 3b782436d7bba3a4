"""The seeded input generator keeps the recipe it is documented with: symmetric A
and B, B an overlap close to I (positive definite, Gershgorin off-diagonal row sums
at most 0.5, so cond(B) <= 3), entries decaying with |i - j|, the workloads' decay
lengths and seeds, determinism per seed, and the batch's log-uniform orders."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("M,ell,seed", [(1, 2.0, 0), (64, 4.0, 7), (300, 6.0, 11), (700, 9.4, 3)])
def test_pair_is_symmetric_and_B_is_a_well_conditioned_overlap(M, ell, seed):
    A, B = synth.banded_pair(M, ell, seed)
    assert A.shape == B.shape == (M, M)
    assert A.dtype == B.dtype == np.float64
    assert np.array_equal(A, A.T) and np.array_equal(B, B.T)
    assert np.all(np.diag(B) == 1.0)
    off = np.abs(B - np.diag(np.diag(B))).sum(axis=1)
    assert off.max() <= 0.5 + 1e-12
    w = np.linalg.eigvalsh(B)
    assert w.min() >= 0.5 - 1e-12 and w.max() <= 1.5 + 1e-12   # Gershgorin
    assert w.max() / w.min() <= 3.0 + 1e-9
    d = np.diag(A)
    assert np.all((d >= -10.0) & (d <= 0.0))


def test_entries_decay_with_the_distance_from_the_diagonal():
    M, ell = 800, 8.0
    A, B = synth.banded_pair(M, ell, 5)
    i, j = np.indices((M, M))
    dist = np.abs(i - j)
    for X in (A - np.diag(np.diag(A)), B - np.eye(M)):
        near = np.abs(X[(dist >= 1) & (dist <= ell)]).mean()
        far = np.abs(X[(dist >= 6 * ell) & (dist <= 7 * ell)]).mean()
        # exp(-6) ~ 2.5e-3 of the near band, within sampling noise
        assert far < 0.02 * near


def test_seeded_and_deterministic():
    A1, B1 = synth.banded_pair(257, 5.0, 42)
    A2, B2 = synth.banded_pair(257, 5.0, 42)
    A3, _ = synth.banded_pair(257, 5.0, 43)
    assert np.array_equal(A1, A2) and np.array_equal(B1, B2)
    assert not np.array_equal(A1, A3)


def test_workload_recipes():
    assert synth.decay_length(512) == pytest.approx(8.0)
    assert synth.decay_length(8192) == pytest.approx(32.0)
    assert synth.decay_length(32768) == pytest.approx(64.0)
    assert synth.SINGLE["m512"] == (512, 8.0, 1)
    assert synth.SINGLE["m8192"] == (8192, 32.0, 2)
    assert synth.SINGLE["m32768"] == (32768, 64.0, 3)
    A, B = synth.workload("m512")
    A0, B0 = synth.banded_pair(512, 8.0, 1)
    assert np.array_equal(A, A0) and np.array_equal(B, B0)


def test_batch_orders_are_log_uniform_in_range():
    sizes = synth.batch_sizes()
    assert len(sizes) == 256
    assert min(sizes) >= 64 and max(sizes) <= 2048
    assert sizes == synth.batch_sizes()
    # log-uniform: about half of the orders below the geometric mean sqrt(64 * 2048)
    below = sum(1 for m in sizes if m < np.sqrt(64 * 2048))
    assert 100 <= below <= 156
