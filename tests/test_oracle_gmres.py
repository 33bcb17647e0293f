"""Pins of the oracle's restarted GMRES and dense far-zone matrix (CPU).

GMRES is checked against facts fixed by the mathematics, not by itself: the
exact solution of small dense systems, termination in at most d steps for a
diagonalizable matrix with d distinct eigenvalues, residual estimates equal
to the explicitly computed residuals, and monotone residuals. The dense
far-zone matrix is checked against the grouped far-zone product.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import gmres as G

A_SIDE, K = 0.25, 2 * np.pi


def _rand(n, seed, shift):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return M / np.sqrt(n) + shift * np.eye(n)


def test_full_length_gmres_is_exact():
    A = _rand(40, 1, 2.0)
    b = W.complex_normal((40,), 2).astype(np.complex128)
    x, hist = G.gmres(lambda v: A @ v, b, restart=40, tol=1e-13, max_steps=40)
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-11
    assert hist[-1] < 1e-12


def test_terminates_in_distinct_eigenvalue_count():
    rng = np.random.default_rng(3)
    n = 30
    Q = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    lam = np.array([1.0 + 1j, 3.0, -2.0 + 0.5j])[rng.integers(0, 3, n)]
    A = Q @ np.diag(lam) @ np.linalg.inv(Q)
    b = W.complex_normal((n,), 4).astype(np.complex128)
    x, hist = G.gmres(lambda v: A @ v, b, restart=30, tol=1e-9, max_steps=30)
    assert len(hist) - 1 <= 3
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) < 1e-8


def test_estimates_are_true_residuals_and_monotone():
    A = _rand(60, 5, 1.5)
    b = W.complex_normal((60,), 6).astype(np.complex128)
    for steps in (1, 4, 9, 17):
        x, hist = G.gmres(lambda v: A @ v, b, restart=60, tol=1e-14, max_steps=steps)
        true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        assert abs(true - hist[-1]) < 1e-10
        assert all(hist[i + 1] <= hist[i] + 1e-14 for i in range(len(hist) - 1))


def test_restarted_gmres_converges_and_reports_true_residual():
    A = _rand(80, 7, 2.5)
    b = W.complex_normal((80,), 8).astype(np.complex128)
    x, hist = G.gmres(lambda v: A @ v, b, restart=5, tol=1e-8, max_steps=200)
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert hist[-1] <= 1e-8 and true <= 1.01e-8
    assert len(hist) - 1 > 5          # it did restart
    assert all(hist[i + 1] <= hist[i] + 1e-14 for i in range(len(hist) - 1))


def test_zero_rhs():
    x, hist = G.gmres(lambda v: 2 * v, np.zeros(5, complex), 5, 1e-6, 10)
    assert not x.any() and hist == [0.0]


@pytest.mark.parametrize("mode", ["ilist", "full"])
def test_far_matrix_matches_grouped_product(mode):
    boxes = W.grid_boxes(3, 3, 4)
    Z = G.far_matrix(boxes, A_SIDE, K, 2, mode)
    x = W.complex_normal((2, len(boxes) * 24), 9).astype(np.complex128)
    y = O.far_mvm(x, boxes, A_SIDE, K, 2, mode=mode)
    assert np.linalg.norm((Z @ x.T).T - y) / np.linalg.norm(y) < 1e-13
    # reciprocity of the operators makes Z^F complex symmetric
    assert np.abs(Z - Z.T).max() <= 1e-12 * np.abs(Z).max()


def test_gmres_on_shifted_far_system():
    boxes = W.grid_boxes(4, 4, 4)
    Z = G.far_matrix(boxes, A_SIDE, K, 2)
    v = W.complex_normal((len(Z),), 10).astype(np.complex128)
    sigma = 2.0 * np.linalg.norm(Z @ v) / np.linalg.norm(v) * np.exp(0.25j * np.pi)
    A = Z + sigma * np.eye(len(Z))
    b = W.complex_normal((len(Z),), 11).astype(np.complex128)
    x, hist = G.gmres(lambda u: sigma * u + O.far_mvm(u[None], boxes, A_SIDE, K, 2)[0],
                      b, restart=100, tol=1e-6, max_steps=200)
    ref = np.linalg.solve(A, b)
    assert hist[-1] <= 1e-6
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-4
