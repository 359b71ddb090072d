"""Pins of the oracle's Band_DFT_Col Part 5 (chemical potential, band energy)
and Part 6 (charge and energy density matrices) against closed forms,
symmetries, limits and invariants that do not restate the oracle's sums."""
import numpy as np
import pytest

import oracle as O


def test_single_level_closed_form():
    # one state holding g electrons: g f(lam - mu) = nelec
    # => mu = lam - kT ln(g / nelec - 1)
    lam, kT, g, ne = 0.37, 0.05, 2.0, 0.6
    mu, eb, cnt, occ = O.fermi([[lam]], [1.0], ne, kT, g)
    assert mu == pytest.approx(lam - kT * np.log(g / ne - 1.0), abs=1e-13)
    assert eb == pytest.approx(ne * lam, abs=1e-13)
    assert cnt == pytest.approx(ne, abs=1e-13)
    assert occ[0, 0] == pytest.approx(ne / g, abs=1e-14)


@pytest.mark.parametrize("kT", [0.3, 0.5, 2.0])
def test_two_levels_half_filled_is_midpoint(kT):
    # f(a) + f(b) = 1 holds exactly at mu = (a + b) / 2 (f(x) + f(-x) = 1)
    a, b = -0.8, 1.3
    mu, eb, cnt, occ = O.fermi([[a, b]], [1.0], 1.0, kT, 1.0)
    assert mu == pytest.approx(0.5 * (a + b), abs=1e-12)
    assert occ[0].sum() == pytest.approx(1.0, abs=1e-13)


def test_symmetric_spectrum_over_weighted_kpoints():
    # a spectrum symmetric about c at every k-point, filled to half its
    # capacity, puts mu at c whatever the weights
    rng = np.random.default_rng(11)
    c, nk, half = 0.25, 3, 7
    x = rng.uniform(0.05, 1.0, (nk, half))
    w = np.sort(np.concatenate([c - x, c + x], axis=1), axis=1)
    wk = np.array([0.2, 0.5, 0.3])
    g = 2.0
    mu, eb, cnt, _ = O.fermi(w, wk, g * 2 * half * wk.sum() / 2, 0.2, g)
    assert mu == pytest.approx(c, abs=1e-12)


def test_zero_temperature_limit_is_sum_of_filled_levels():
    # a gap of 1 at kT = 1e-3: occupations are 1 below and 0 above to
    # within exp(-500); the band energy is g times the weighted sum of the
    # filled levels and mu lies in the gap
    rng = np.random.default_rng(5)
    nk, n, nfill = 4, 10, 6
    lowv = rng.uniform(-2.0, -0.5, (nk, nfill))
    highv = rng.uniform(0.5, 2.0, (nk, n - nfill))
    w = np.sort(np.concatenate([lowv, highv], axis=1), axis=1)
    wk = np.full(nk, 1.0 / nk)
    g = 2.0
    mu, eb, cnt, occ = O.fermi(w, wk, g * nfill, 1e-3, g)
    assert -0.5 < mu < 0.5
    assert eb == pytest.approx(g * (wk[:, None] * w[:, :nfill]).sum(), abs=1e-12)
    assert np.array_equal(occ > 0.5, np.arange(n)[None, :].repeat(nk, 0) < nfill)


def test_shift_and_scale_covariance():
    rng = np.random.default_rng(8)
    w = np.sort(rng.uniform(-1, 1, (2, 9)), axis=1)
    wk = [0.4, 0.6]
    mu0, eb0, _, _ = O.fermi(w, wk, 7.0, 0.15, 2.0)
    mu1, eb1, _, _ = O.fermi(w + 0.75, wk, 7.0, 0.15, 2.0)
    assert mu1 == pytest.approx(mu0 + 0.75, abs=1e-12)
    assert eb1 == pytest.approx(eb0 + 0.75 * 7.0, abs=1e-11)
    mu2, eb2, _, _ = O.fermi(3.0 * w, wk, 7.0, 0.45, 2.0)
    assert mu2 == pytest.approx(3.0 * mu0, abs=1e-11)
    assert eb2 == pytest.approx(3.0 * eb0, abs=1e-11)


def test_invalid_arguments():
    with pytest.raises(ValueError):
        O.fermi([[0.0, 1.0]], [1.0], 1.0, 0.0, 2.0)      # kT = 0
    with pytest.raises(ValueError):
        O.fermi([[0.0, 1.0]], [1.0], 4.0, 0.1, 2.0)      # nelec = capacity


def _s_orthonormal(n, nk, rng):
    """S (Hermitian positive definite) and nk matrices C_k with C^H S C = I:
    C = L^{-H} Q with S = L L^H and Q unitary."""
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    S = np.eye(n) + 0.2 * (A + A.conj().T)
    L = np.linalg.cholesky(S)
    Cs = []
    for _ in range(nk):
        Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        Q, R = np.linalg.qr(Z)
        Cs.append(np.linalg.solve(L.conj().T, Q))
    return S, np.array(Cs)


def test_density_traces_count_electrons_and_band_energy():
    # tr(rho S) = g sum_k wk sum_j f_kj and tr(E S) = E_band because every
    # C_k is S-orthonormal
    rng = np.random.default_rng(3)
    n, nk = 9, 3
    S, C = _s_orthonormal(n, nk, rng)
    w = np.sort(rng.uniform(-1, 1, (nk, n)), axis=1)
    wk = np.array([0.5, 0.3, 0.2])
    g = 2.0
    mu, eb, cnt, occ = O.fermi(w, wk, 8.0, 0.2, g)
    rho, E = O.density(C, w, occ, wk, g)
    assert np.trace(rho @ S).real == pytest.approx(cnt, abs=1e-12)
    assert abs(np.trace(rho @ S).imag) < 1e-12
    assert np.trace(E @ S).real == pytest.approx(eb, abs=1e-12)
    assert np.abs(rho - rho.conj().T).max() < 1e-15
    assert np.linalg.eigvalsh(rho).min() > -1e-13


def test_density_idempotent_for_integer_occupations():
    # one k-point, g = 1, f in {0, 1}: rho S rho = rho (S-orthogonal projector)
    rng = np.random.default_rng(4)
    n = 8
    S, C = _s_orthonormal(n, 1, rng)
    occ = np.zeros((1, n))
    occ[0, :5] = 1.0
    w = np.sort(rng.uniform(-1, 1, (1, n)), axis=1)
    rho, E = O.density(C, w, occ, [1.0], 1.0)
    assert np.abs(rho @ S @ rho - rho).max() < 1e-12
    # the energy density matrix is rho with the filled levels as weights
    assert np.abs(E @ S @ rho - E).max() < 1e-12


def test_density_truncated_columns_agree():
    rng = np.random.default_rng(6)
    n, nk, nocc = 7, 2, 4
    _, C = _s_orthonormal(n, nk, rng)
    w = np.sort(rng.uniform(-1, 1, (nk, n)), axis=1)
    occ = rng.uniform(0, 1, (nk, n))
    occ[:, nocc:] = 0.0
    r1, e1 = O.density(C, w, occ, [0.5, 0.5], 2.0)
    r2, e2 = O.density(C, w, occ, [0.5, 0.5], 2.0, nocc=nocc)
    assert np.abs(r1 - r2).max() < 1e-15 and np.abs(e1 - e2).max() < 1e-15


def test_density_entries_match_full_matrices():
    rng = np.random.default_rng(12)
    n, nk = 11, 2
    _, C = _s_orthonormal(n, nk, rng)
    w = np.sort(rng.uniform(-1, 1, (nk, n)), axis=1)
    occ = rng.uniform(0, 1, (nk, n))
    wk = [0.3, 0.7]
    rho, E = O.density(C, w, occ, wk, 2.0)
    pairs = [(0, 0), (5, 2), (10, 9), (3, 3), (10, 0)]
    r, e = O.density_entries(np.transpose(C, (0, 2, 1)), w, occ, wk, 2.0, pairs)
    for q, (a, b) in enumerate(pairs):
        assert r[q] == rho[a, b] and e[q] == E[a, b]

