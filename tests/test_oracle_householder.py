"""Pins for the oracle's Householder tridiagonalisation (Section III,
Procedures 1-6 of Eigen_HH) and its back-transformation ("rearrangement of
eigenvectors").  Each check is fixed by mathematics, not by the oracle."""
import numpy as np
import pytest

import oracle as O


def rand_herm(rng, n):
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return (A + A.conj().T) / 2


def tri(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64, 130])
def test_similarity_invariants(n):
    rng = np.random.default_rng(n)
    A = rand_herm(rng, n)
    d, e, tau, V = O.zhetrd(A)
    T = tri(d, e)
    eps = np.finfo(float).eps
    # trace and Frobenius norm are unitary invariants
    assert abs(np.trace(T) - np.trace(A).real) <= 10 * n * eps * np.linalg.norm(A)
    assert abs(np.linalg.norm(T) - np.linalg.norm(A)) <= 10 * n * eps * np.linalg.norm(A)
    # Q = H_0 ... H_{n-2} is unitary and Q T Q^H = A
    Q = O.apply_q(V, tau, np.eye(n))
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() <= 10 * n * eps
    assert np.linalg.norm(Q @ T @ Q.conj().T - A) <= 10 * n * eps * np.linalg.norm(A)
    # the spectrum is preserved (LAPACK as a third opinion)
    assert np.allclose(np.linalg.eigvalsh(T), np.linalg.eigvalsh(A), atol=50 * n * eps * np.linalg.norm(A))


@pytest.mark.parametrize("a21", [3 + 4j, -3 + 4j, 2.0 + 0j, -2.0 + 0j, 0.5j])
def test_two_by_two_is_a_phase_fix(a21):
    # n = 2: one reflector of length 1; T = [[a11, beta], [beta, a22]],
    # beta = -sign(Re a21) |a21| (sign(0) = +1) and H^H x = beta e_1, except
    # that a real a21 needs no reflector at all.
    A = np.array([[1.5, np.conj(a21)], [a21, -0.25]])
    d, e, tau, V = O.zhetrd(A)
    assert np.allclose(d, [1.5, -0.25], atol=1e-15)
    t = tau[0]
    if a21.imag == 0:
        # already real: no reflection (tau = 0) and e = a21
        assert t == 0 and e[0] == a21.real
        return
    sgn = 1.0 if a21.real >= 0 else -1.0
    assert e[0] == pytest.approx(-sgn * abs(a21), abs=1e-15)
    # H = I - tau v v^H with v = [1]; H^H x = (1 - conj(tau)) a21 = beta
    assert abs((1 - np.conj(t)) * a21 - e[0]) <= 1e-14
    assert abs(abs(1 - t) - 1.0) <= 1e-14          # a unit-modulus phase


def test_real_tridiagonal_input_is_unchanged_up_to_sign():
    rng = np.random.default_rng(7)
    n = 12
    d0 = rng.standard_normal(n)
    e0 = rng.standard_normal(n - 1)
    d, e, tau, V = O.zhetrd(tri(d0, e0).astype(complex))
    assert np.allclose(d, d0, atol=1e-15)
    assert np.allclose(np.abs(e), np.abs(e0), atol=1e-15)


def test_zero_column_gives_identity_reflector():
    # a column that is already reduced takes tau = 0 (H = I)
    A = np.diag([1.0, 2.0, 3.0]).astype(complex)
    d, e, tau, V = O.zhetrd(A)
    assert np.all(tau == 0)
    assert np.allclose(d, [1, 2, 3]) and np.allclose(e, 0)


def test_reflector_annihilates_its_column():
    # H_i^H maps the column below the diagonal onto beta e_1 (Procedure 2)
    rng = np.random.default_rng(3)
    n = 9
    A = rand_herm(rng, n)
    d, e, tau, V = O.zhetrd(A)
    x = A[1:, 0]
    v = V[1:, 0]
    Hh = np.eye(n - 1) - np.conj(tau[0]) * np.outer(v, v.conj())
    y = Hh @ x
    assert abs(y[0] - e[0]) <= 1e-13 and np.abs(y[1:]).max() <= 1e-13
    assert v[0] == 1


def test_back_transform_gives_eigenvectors():
    rng = np.random.default_rng(11)
    n = 40
    A = rand_herm(rng, n)
    d, e, tau, V = O.zhetrd(A)
    w, Z = O.tridiag_ql(d, e)
    U = O.apply_q(V, tau, Z.astype(complex))
    eps = np.finfo(float).eps
    assert np.linalg.norm(A @ U - U * w) <= 20 * n * eps * np.linalg.norm(A)
    assert np.abs(U.conj().T @ U - np.eye(n)).max() <= 20 * n * eps


def test_zgemm_matches_definition():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((7, 5)) + 1j * rng.standard_normal((7, 5))
    B = rng.standard_normal((5, 6)) + 1j * rng.standard_normal((5, 6))
    C0 = rng.standard_normal((7, 6)) + 1j * rng.standard_normal((7, 6))
    got = O.zgemm("N", "N", A, B, alpha=2 - 1j, beta=0.5j, C=C0)
    assert np.allclose(got, (2 - 1j) * A @ B + 0.5j * C0, atol=1e-13)
    got = O.zgemm("C", "N", A, A)
    assert np.allclose(got, A.conj().T @ A, atol=1e-13)
    got = O.zgemm("N", "C", B, B)
    assert np.allclose(got, B @ B.conj().T, atol=1e-13)


def test_normalize_cols_unit_norm_same_direction():
    # Eigen_HH's normalisation: every column leaves with unit 2-norm and
    # points the same way as it came in (a 3-4-5 triangle, then columns whose
    # norms span twelve orders of magnitude)
    eps = np.finfo(float).eps
    got = O.normalize_cols(np.array([[3.0], [4.0j]]))
    assert np.abs(got - np.array([[0.6], [0.8j]])).max() <= 2 * eps
    rng = np.random.default_rng(13)
    U = (rng.standard_normal((9, 6)) + 1j * rng.standard_normal((9, 6))) * np.logspace(-6, 6, 6)
    got = O.normalize_cols(U)
    assert np.abs(np.linalg.norm(got, axis=0) - 1.0).max() <= 8 * eps
    for j in range(U.shape[1]):
        u = U[:, j] / np.linalg.norm(U[:, j])
        assert abs(abs(np.vdot(u, got[:, j])) - 1.0) <= 8 * eps
        assert np.abs(got[:, j] - u).max() <= 8 * eps
