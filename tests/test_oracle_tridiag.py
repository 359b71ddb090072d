"""Pins for the oracle's tridiagonal eigensolver (the LAPACK step of
Eigen_HH, Section III): closed-form spectra, Sturm counts, bisection."""
import math

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("n", [1, 2, 5, 33, 100])
def test_toeplitz_closed_form(n):
    # tridiag(b, a, b): l_j = a + 2 b cos(j pi/(n+1)),
    # z_j(i) = sqrt(2/(n+1)) sin(i j pi/(n+1))  (i, j = 1..n)
    a, b = 0.3, -1.7
    d = np.full(n, a)
    e = np.full(n - 1, b)
    w, Z = O.tridiag_ql(d, e)
    j = np.arange(1, n + 1)
    exact = np.sort(a + 2 * b * np.cos(j * np.pi / (n + 1)))
    assert np.abs(w - exact).max() <= 8 * n * np.finfo(float).eps * 4
    # eigenvectors up to sign
    for q in range(n):
        lam = w[q]
        jj = np.argmin(np.abs(a + 2 * b * np.cos(j * np.pi / (n + 1)) - lam))
        zex = math.sqrt(2.0 / (n + 1)) * np.sin(np.arange(1, n + 1) * j[jj] * np.pi / (n + 1))
        assert abs(abs(zex @ Z[:, q]) - 1.0) <= 1e-12


@pytest.mark.parametrize("n", [2, 7, 50, 201])
def test_clement_integer_spectrum(n):
    # Clement (Kac) matrix: zero diagonal, off-diagonal sqrt(i (n - i)),
    # eigenvalues -(n-1), -(n-3), ..., n-1.
    d = np.zeros(n)
    e = np.sqrt(np.arange(1, n) * (n - np.arange(1, n)))
    w, Z = O.tridiag_ql(d, e)
    exact = np.arange(-(n - 1), n, 2, dtype=float)
    assert np.abs(w - exact).max() <= 50 * n * np.finfo(float).eps
    wb = O.bisect_eigs(d, e)
    assert np.abs(wb - exact).max() <= 50 * n * np.finfo(float).eps
    # Sturm counts are integers fixed exactly away from the eigenvalues
    for x, cnt in [(exact[0] - 0.5, 0), (exact[-1] + 0.5, n)] + [(exact[i] + 1.0, i + 1) for i in range(n - 1)]:
        assert O.sturm_count(d, e, x) == cnt


def test_ql_vectors_orthonormal_and_residual():
    rng = np.random.default_rng(2)
    n = 300
    d = rng.standard_normal(n)
    e = rng.standard_normal(n - 1)
    w, Z = O.tridiag_ql(d, e)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    eps = np.finfo(float).eps
    assert np.all(np.diff(w) >= 0)
    assert np.linalg.norm(T @ Z - Z * w) <= 20 * n * eps * np.linalg.norm(T)
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 20 * n * eps
    assert np.abs(O.bisect_eigs(d, e) - w).max() <= 4 * n * eps * np.abs(w).max()


def test_wilkinson_close_pairs():
    # W_21^+: eigenvalue pairs agree to ~1e-14 -- a hard case for accuracy
    n = 21
    d = np.abs(np.arange(n) - 10).astype(float)
    e = np.ones(n - 1)
    w, Z = O.tridiag_ql(d, e)
    ref = np.linalg.eigvalsh(np.diag(d) + np.diag(e, 1) + np.diag(e, -1))
    assert np.abs(w - ref).max() <= 1e-13
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-13


def test_values_only_matches_vectors_run():
    rng = np.random.default_rng(4)
    d = rng.standard_normal(64)
    e = rng.standard_normal(63)
    w1, _ = O.tridiag_ql(d, e, vectors=False)
    w2, _ = O.tridiag_ql(d, e, vectors=True)
    assert np.array_equal(w1, w2)
