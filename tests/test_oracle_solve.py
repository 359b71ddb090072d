"""Pins for the oracle's whole per-k solve (Band_DFT_Col Parts 2-4,
Section III): closed forms, known spectra, invariances, inertia, brute force,
hand-derived fixtures, error statuses, and LAPACK as a third opinion."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from paper_1402_4247_amd import inputs as G

EPS = np.finfo(float).eps
HERE = os.path.dirname(os.path.abspath(__file__))


def checks(H, S, w, C):
    """r_res (Frobenius), r_orth (max entry) and per-column backward error."""
    r_res = np.linalg.norm(H @ C - S @ C * w) / np.linalg.norm(H)
    r_orth = np.abs(C.conj().T @ S @ C - np.eye(len(w))).max()
    return r_res, r_orth


def rand_herm(rng, n, scale=1.0):
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return scale * (A + A.conj().T) / 2


def rand_spd(rng, n):
    B = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2 * n)
    return np.eye(n) + 0.3 * (B @ B.conj().T)


def load_fixture_matrix(rows):
    return np.array([[complex(re, im) for re, im in row] for row in rows])


def test_hand_fixtures():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        H = load_fixture_matrix(c["H"])
        S = load_fixture_matrix(c["S"])
        st, w, C = O.solve_k(H, S)
        assert st == O.OK, c["name"]
        assert np.allclose(w, c["eigenvalues"], atol=1e-14, rtol=0), c["name"]
        r_res, r_orth = checks(H, S, w, C)
        assert r_res <= 1e-14 and r_orth <= 1e-14, c["name"]


def test_one_by_one():
    H = np.array([[-3.0 + 0.7j]])       # imaginary part of the diagonal is ignored
    S = np.array([[4.0]])
    st, w, C = O.solve_k(H, S)
    assert st == O.OK
    assert w[0] == pytest.approx(-0.75, abs=1e-16)
    assert abs(abs(C[0, 0]) - 0.5) <= 1e-16


@pytest.mark.parametrize("seed", range(6))
def test_two_by_two_generalized_quadratic(seed):
    # det(H - l S) = 0:
    # l^2 (s11 s22 - |s12|^2) - l (h11 s22 + h22 s11 - 2 Re(h12 conj(s12)))
    #   + (h11 h22 - |h12|^2) = 0
    rng = np.random.default_rng(100 + seed)
    H = rand_herm(rng, 2)
    S = rand_spd(rng, 2)
    a = (S[0, 0] * S[1, 1] - abs(S[0, 1]) ** 2).real
    b = -(H[0, 0] * S[1, 1] + H[1, 1] * S[0, 0] - 2 * (H[0, 1] * np.conj(S[0, 1])).real).real
    c = (H[0, 0] * H[1, 1] - abs(H[0, 1]) ** 2).real
    disc = math.sqrt(b * b - 4 * a * c)
    q = -0.5 * (b + math.copysign(disc, b))             # stable quadratic formula
    roots = sorted([q / a, c / q])
    st, w, C = O.solve_k(H, S)
    assert st == O.OK
    assert np.allclose(w, roots, atol=1e-14 * max(1, abs(roots[0]), abs(roots[1])))


@pytest.mark.parametrize("seed", range(6))
def test_three_by_three_trigonometric(seed):
    # Smith (1961): eigenvalues of a 3x3 Hermitian matrix in closed form
    rng = np.random.default_rng(200 + seed)
    A = rand_herm(rng, 3)
    q = np.trace(A).real / 3
    p1 = abs(A[0, 1]) ** 2 + abs(A[0, 2]) ** 2 + abs(A[1, 2]) ** 2
    p2 = sum((A[i, i].real - q) ** 2 for i in range(3)) + 2 * p1
    p = math.sqrt(p2 / 6)
    B = (A - q * np.eye(3)) / p
    detB = (B[0, 0] * (B[1, 1] * B[2, 2] - B[1, 2] * B[2, 1])
            - B[0, 1] * (B[1, 0] * B[2, 2] - B[1, 2] * B[2, 0])
            + B[0, 2] * (B[1, 0] * B[2, 1] - B[1, 1] * B[2, 0])).real
    r = max(-1.0, min(1.0, detB / 2))
    phi = math.acos(r) / 3
    l1 = q + 2 * p * math.cos(phi)
    l3 = q + 2 * p * math.cos(phi + 2 * math.pi / 3)
    l2 = 3 * q - l1 - l3
    st, w, C = O.solve_k(A, np.eye(3))
    assert st == O.OK
    assert np.allclose(w, sorted([l1, l2, l3]), atol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_brute_force_determinant_roots(n):
    # roots of det(H - l S), the polynomial fixed by its values at n+1 points
    rng = np.random.default_rng(300 + n)
    H = rand_herm(rng, n)
    S = rand_spd(rng, n)
    xs = np.linspace(-4, 4, n + 1)
    vals = [np.linalg.det(H - x * S).real for x in xs]
    coef = np.linalg.solve(np.vander(xs, n + 1), vals)
    roots = np.sort(np.roots(coef).real)
    st, w, C = O.solve_k(H, S)
    assert st == O.OK
    assert np.allclose(w, roots, atol=1e-9)


@pytest.mark.parametrize("n", [16, 97])
def test_known_spectrum(n):
    rng = np.random.default_rng(400 + n)
    lam = np.sort(rng.uniform(-2, 2, n))
    Q = G.haar_unitary(rng, n)
    H = (Q * lam) @ Q.conj().T
    st, w, C = O.solve_k(H, np.eye(n))
    assert st == O.OK and np.abs(w - lam).max() <= 100 * n * EPS
    # generalized: H = B Q L Q^H B^H, S = B B^H
    B = np.linalg.cholesky(rand_spd(rng, n))
    H2 = B @ H @ B.conj().T
    S2 = B @ B.conj().T
    st, w, C = O.solve_k(H2, S2)
    assert st == O.OK and np.abs(w - lam).max() <= 200 * n * EPS
    r_res, r_orth = checks(H2, S2, w, C)
    assert r_res <= 1e-13 and r_orth <= 1e-13


def test_invariances():
    rng = np.random.default_rng(9)
    n = 24
    H = rand_herm(rng, n)
    S = rand_spd(rng, n)
    st, w, C = O.solve_k(H, S)
    assert st == O.OK
    tol = 1e-12
    # shift: (H + sigma S, S) -> l + sigma
    _, w2, _ = O.solve_k(H + 0.75 * S, S)
    assert np.abs(w2 - (w + 0.75)).max() <= tol
    # scale H: -> alpha l (alpha > 0 keeps the order)
    _, w2, _ = O.solve_k(3.0 * H, S)
    assert np.abs(w2 - 3.0 * w).max() <= tol
    # scale S: -> l / beta, C / sqrt(beta)
    _, w2, C2 = O.solve_k(H, 2.0 * S)
    assert np.abs(w2 - w / 2.0).max() <= tol
    assert np.allclose(np.abs(C2), np.abs(C) / math.sqrt(2.0), atol=1e-10)
    # diagonal unitary gauge: (D H D^H, D S D^H) -> same l, |D C| = |C|
    D = np.exp(1j * rng.uniform(0, 2 * np.pi, n))
    _, w2, C2 = O.solve_k(D[:, None] * H * D.conj()[None, :], D[:, None] * S * D.conj()[None, :])
    assert np.abs(w2 - w).max() <= tol
    assert np.allclose(np.abs(C2), np.abs(C), atol=1e-10)
    # permutation of the basis -> same l
    p = rng.permutation(n)
    _, w2, _ = O.solve_k(H[np.ix_(p, p)], S[np.ix_(p, p)])
    assert np.abs(w2 - w).max() <= tol
    # block diagonal -> union of spectra
    H2 = rand_herm(rng, 10)
    S2 = rand_spd(rng, 10)
    _, wb, _ = O.solve_k(H2, S2)
    Hb = sl.block_diag(H, H2)
    Sb = sl.block_diag(S, S2)
    _, wu, _ = O.solve_k(Hb, Sb)
    assert np.abs(wu - np.sort(np.concatenate([w, wb]))).max() <= tol


def test_sylvester_inertia():
    # #{l_j < sigma} = number of negative eigenvalues of H - sigma S, counted
    # from the block-diagonal factor of an LDL^H factorisation
    rng = np.random.default_rng(12)
    n = 40
    H = rand_herm(rng, n)
    S = rand_spd(rng, n)
    st, w, C = O.solve_k(H, S)
    for sigma in [-3.0, -0.4, 0.1, 1.3, 5.0]:
        lu, dblk, perm = sl.ldl(H - sigma * S, lower=True, hermitian=True)
        neg = int(np.sum(np.linalg.eigvalsh(dblk) < 0))
        assert int(np.sum(w < sigma)) == neg


@pytest.mark.parametrize("gen", ["config1", "config2_128"])
def test_residuals_and_third_opinion(gen):
    if gen == "config1":
        H, S = G.config1(128, 1001)
    else:
        Hs, Ss = G.config2(128, 1, 2002)
        H, S = Hs[0], Ss[0]
    st, w, C, stg = O.solve_k(H, S, stages=True)
    assert st == O.OK
    r_res, r_orth = checks(H, S, w, C)
    assert r_res <= 1e-12 and r_orth <= 1e-12
    wl = sl.eigh(H, S, eigvals_only=True)
    assert np.abs(w - wl).max() <= 1e-10 * np.abs(wl).max()
    # stage pins: X^H S X = I, eig(A) = eig(H, S), T_S similar to S
    X = stg["X"]
    assert np.abs(X.conj().T @ S @ X - np.eye(len(w))).max() <= 1e-12
    assert np.abs(np.linalg.eigvalsh(stg["A"]) - wl).max() <= 1e-10 * np.abs(wl).max()
    assert np.allclose(np.sort(stg["s"]), np.linalg.eigvalsh(S), atol=1e-13)


def test_layout_trap_nonreal_hermitian():
    # A row-major matrix read as column-major is conj(H): the residual with
    # conj(C) is large, with C small.
    H, S = G.config1(32, 5)
    st, w, C = O.solve_k(H, S)
    r_res, _ = checks(H, S, w, C)
    bad, _ = checks(H, S, w, C.conj())
    assert r_res <= 1e-13 and bad > 1e-3


def test_error_statuses():
    n = 6
    H = np.diag(np.arange(n, dtype=float)).astype(complex)
    S = np.eye(n, dtype=complex)
    S[n - 1, n - 1] = -1.0
    st, _, _ = O.solve_k(H, S)
    assert st == O.ENOTPD
    S = np.eye(n, dtype=complex)
    S[n - 1, n - 1] = 1e-14                  # below s_tol * s_max
    st, _, _ = O.solve_k(H, S)
    assert st == O.ENOTPD
    Hn = H.copy()
    Hn[3, 1] = np.nan
    st, _, _ = O.solve_k(Hn, np.eye(n))
    assert st == O.ENONFINITE
    Hn = H.copy()
    Hn[1, 3] = np.nan                         # upper triangle is never read
    st, _, _ = O.solve_k(Hn, np.eye(n))
    assert st == O.OK


def test_values_only_equals_vectors_eigenvalues():
    H, S = G.config1(48, 77)
    st1, w1, _ = O.solve_k(H, S, vectors=False)
    st2, w2, _ = O.solve_k(H, S, vectors=True)
    assert st1 == st2 == O.OK and np.array_equal(w1, w2)


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
def test_known_spectrum_ill_conditioned_overlap(kappa):
    # S = U diag(s) U^H with kappa(S) = kappa and known generalized eigenpairs:
    # the eigenvalues must lie within the first-order perturbation bound
    # 4 n eps (||H|| + |lambda| ||S||) ||c_j||^2 of the exact ones
    n = 120
    H, S, lam, Cex = G.known_spectrum_pencil(n, kappa, 31)
    eps = np.finfo(float).eps
    tol = 4 * n * eps * (np.linalg.norm(H, 2) + np.abs(lam) * np.linalg.norm(S, 2)) * np.linalg.norm(Cex, axis=0) ** 2
    st, w, C = O.solve_k(H, S)
    assert st == 0
    assert np.all(np.abs(w - lam) <= tol)
    assert np.abs(C.conj().T @ S @ C - np.eye(n)).max() <= 4 * n * eps * kappa
    assert np.linalg.norm(H @ C - S @ C * w) / np.linalg.norm(H) <= 4 * n * eps * kappa
