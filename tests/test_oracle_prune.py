"""Pins of the oracle's pruned canonical orthogonalisation (Part 2 variant):
no pruning reproduces the paper's form, a diagonal pencil with zero overlap
directions has a closed form, the result is invariant under a unitary change
of basis, and for S of rank r the kept eigenvalues are those of the pencil
restricted to range(S) (LAPACK as a third opinion)."""
import numpy as np
import scipy.linalg

import oracle as O


def _herm(rng, n, scale=1.0):
    B = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return scale * (B + B.conj().T) / 2


def test_no_pruning_equals_paper_form():
    rng = np.random.default_rng(1)
    n = 24
    H = _herm(rng, n)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    S = np.eye(n) + 0.2 * (A + A.conj().T)
    st, m, w, C = O.solve_k_prune(H, S)
    st0, w0, C0 = O.solve_k(H, S)
    assert st == 0 and st0 == 0 and m == n
    assert np.array_equal(w, w0) and np.array_equal(C, C0)


def test_diagonal_pencil_with_null_directions():
    h = np.array([3.0, -1.0, 2.0, 5.0, 0.5, -4.0])
    s = np.array([2.0, 1.0, 0.0, 4.0, 1e-20, 0.5])
    st, m, w, C = O.solve_k_prune(np.diag(h).astype(complex), np.diag(s).astype(complex))
    keep = s > 1e-12 * s.max()
    assert st == 0 and m == keep.sum()
    assert np.allclose(w[:m], np.sort(h[keep] / s[keep]), rtol=0, atol=1e-14)
    assert np.all(np.isinf(w[m:])) and np.all(C[:, m:] == 0)
    # C' is S-orthonormal on the kept space
    S = np.diag(s)
    Ck = C[:, :m]
    assert np.abs(Ck.conj().T @ S @ Ck - np.eye(m)).max() < 1e-14


def test_unitary_invariance():
    rng = np.random.default_rng(2)
    n, r = 20, 15
    B = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    S = B @ B.conj().T
    H = _herm(rng, n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    st1, m1, w1, _ = O.solve_k_prune(H, S, s_tol=1e-10)
    st2, m2, w2, _ = O.solve_k_prune(Q @ H @ Q.conj().T, Q @ S @ Q.conj().T, s_tol=1e-10)
    assert st1 == 0 and st2 == 0 and m1 == m2 == r
    assert np.abs(w1[:r] - w2[:r]).max() < 1e-9 * np.abs(w1[:r]).max()


def test_rank_deficient_overlap_matches_restricted_pencil():
    rng = np.random.default_rng(3)
    n, r = 30, 22
    B = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    S = B @ B.conj().T
    H = _herm(rng, n)
    st, m, w, C = O.solve_k_prune(H, S, s_tol=1e-10)
    P, _ = np.linalg.qr(B)                      # orthonormal basis of range(S)
    ref = scipy.linalg.eigh(P.conj().T @ H @ P, P.conj().T @ S @ P, eigvals_only=True)
    assert st == 0 and m == r
    assert np.abs(w[:m] - ref).max() < 1e-9 * np.abs(ref).max()
    # the kept pairs satisfy the Galerkin condition on range(S) (the full
    # residual need not vanish: H c has components S c lambda cannot match)
    Ck = C[:, :m]
    assert np.linalg.norm(P.conj().T @ (H @ Ck - S @ Ck * w[:m])) / np.linalg.norm(H) < 1e-10
    assert np.abs(Ck.conj().T @ S @ Ck - np.eye(m)).max() < 1e-10
