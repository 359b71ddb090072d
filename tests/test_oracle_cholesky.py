"""Pins of the oracle's Part 2 variant (Cholesky factor S = L L^H and its
inverse, X = L^{-H}): reconstruction, uniqueness of the factor, 1x1 and 2x2
closed forms, rejection of indefinite and near-singular S, and the pencil's
eigenvalues through L^{-1} H L^{-H}."""
import numpy as np

import oracle as O


def test_cholesky_reconstructs_and_is_unique():
    rng = np.random.default_rng(21)
    for n in (1, 2, 7, 40):
        A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
        S = np.eye(n) + 0.3 * (A + A.conj().T)
        st, L, Li = O.cholesky_inv(np.tril(S))          # only the lower triangle is read
        assert st == 0
        assert np.abs(np.triu(L, 1)).max() == 0.0 and np.abs(np.triu(Li, 1)).max() == 0.0
        d = np.diag(L)
        assert np.all(d.real > 0) and np.all(d.imag == 0)
        assert np.abs(L @ L.conj().T - S).max() < 1e-14 * n
        assert np.abs(Li @ L - np.eye(n)).max() < 1e-13 * n
        # X = L^{-H} is an S-orthonormaliser
        X = Li.conj().T
        assert np.abs(X.conj().T @ S @ X - np.eye(n)).max() < 1e-13 * n


def test_cholesky_closed_forms():
    # 1 x 1: L = sqrt(s); 2 x 2 Hermitian with known factor
    st, L, Li = O.cholesky_inv(np.array([[4.0 + 0j]]))
    assert st == 0 and L[0, 0] == 2.0 and Li[0, 0] == 0.5
    a, b, c = 9.0, 3.0 - 6.0j, 14.0           # S = [[a, conj(b)], [b, c]]
    S = np.array([[a, np.conj(b)], [b, c]])
    st, L, Li = O.cholesky_inv(S)
    l11 = 3.0
    l21 = b / l11
    l22 = np.sqrt(c - abs(l21) ** 2)
    assert st == 0
    assert abs(L[0, 0] - l11) < 1e-15 and abs(L[1, 0] - l21) < 1e-15 and abs(L[1, 1] - l22) < 1e-15


def test_cholesky_rejects_indefinite_and_near_singular():
    st, _, _ = O.cholesky_inv(np.array([[1.0, 2.0], [2.0, 1.0]], dtype=complex))
    assert st == O.ENOTPD
    S = np.array([[1.0, 1.0], [1.0, 1.0 + 1e-14]], dtype=complex)
    st, _, _ = O.cholesky_inv(S, s_tol=1e-12)
    assert st == O.ENOTPD


def test_cholesky_orthonormaliser_gives_same_pencil_eigenvalues():
    # eig(L^{-1} H L^{-H}) = eig(H, S): same eigenvalues as the paper's form
    rng = np.random.default_rng(22)
    n = 30
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    S = np.eye(n) + 0.2 * (A + A.conj().T)
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = (B + B.conj().T) / 2
    st, L, Li = O.cholesky_inv(S)
    At = Li @ H @ Li.conj().T
    st2, w0, _ = O.solve_k(H, S)
    assert st == 0 and st2 == 0
    assert np.abs(np.linalg.eigvalsh((At + At.conj().T) / 2) - w0).max() < 1e-12 * np.abs(w0).max()
