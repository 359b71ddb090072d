"""Stage parity on the GPU: Householder tridiagonalisation (Procedures 1-6),
the divide-and-conquer tridiagonal eigensolver and the back-transformation
("rearrangement of eigenvectors"), each against the oracle on the same
seeded inputs, at sizes spanning several 64-row tiles and 32-column panels
with ragged tails."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, EPS, K, check, dev, host

pytestmark = pytest.mark.gpu


def mx(a):
    a = np.asarray(a)
    return float(np.abs(a).max()) if a.size else 0.0


def rand_herm(rng, n):
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return (A + A.conj().T) / 2


def gpu_hetrd(As, nb=0):
    kg = K()
    nk, n = As.shape[0], As.shape[1]
    dA = dev(As)
    dd = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    de = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    dtau = torch.zeros((nk, n), dtype=torch.complex128, device=DEV)
    dV = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    with kg.Context(0) as ctx:
        check(kg.hetrd_device(ctx, dA, n, n, nk, dd, de, dtau, dV, opts=kg.make_opts(panel_nb=nb)), "hetrd")
        torch.cuda.synchronize()
    return dd.cpu().numpy(), de.cpu().numpy(), dtau.cpu().numpy(), host(dV)


# n <= 128 runs entirely in the LDS-resident tail kernel; larger n hands over
# to it at the first panel start whose trailing order is at most 128
@pytest.mark.parametrize("n,nb", [(1, 0), (2, 0), (3, 0), (17, 0), (64, 0), (65, 0), (128, 0), (129, 0), (130, 0),
                                  (161, 0), (200, 0), (200, 8), (97, 64), (250, 24), (300, 48)])
def test_hetrd_matches_oracle(n, nb):
    rng = np.random.default_rng(n + 7 * nb)
    nk = 2
    As = np.stack([rand_herm(rng, n) for _ in range(nk)])
    d, e, tau, V = gpu_hetrd(As, nb)
    for q in range(nk):
        A = As[q]
        nf = np.linalg.norm(A)
        d0, e0, tau0, V0 = O.zhetrd(A)
        tol = 64 * n * EPS * nf
        assert mx(d[q] - d0) <= tol, f"d k={q}: {mx(d[q]-d0)}"
        assert mx(e[q, : n - 1] - e0) <= tol, f"e k={q}: {mx(e[q, : n - 1] - e0)}"
        # same reflector convention -> same tau and v up to rounding
        assert mx(tau[q, : n - 1] - tau0) <= 64 * n * EPS * 4, f"tau: {mx(tau[q, : n - 1] - tau0)}"
        assert mx(V[q] - V0) <= 64 * n * EPS * 16, f"V: {mx(V[q] - V0)}"
        # similarity: spectrum of the GPU T equals that of A
        wg = O.bisect_eigs(d[q], e[q, : n - 1])
        assert mx(wg - np.sort(np.linalg.eigvalsh(A))) <= tol


def gpu_stedc(ds, es):
    kg = K()
    nk, n = ds.shape
    dd = torch.from_numpy(np.ascontiguousarray(ds)).to(DEV)
    de = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    de[:, : n - 1] = torch.from_numpy(np.ascontiguousarray(es)).to(DEV)
    dw = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    dZ = torch.zeros((nk, n, n), dtype=torch.float64, device=DEV)
    st = torch.zeros(nk, dtype=torch.int32, device=DEV)
    with kg.Context(0) as ctx:
        check(kg.stedc_device(ctx, dd, de, n, nk, dw, dZ, st), "stedc")
        torch.cuda.synchronize()
    return dw.cpu().numpy(), np.swapaxes(dZ.cpu().numpy(), -1, -2), st.cpu().numpy()


def tri(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def stedc_cases():
    rng = np.random.default_rng(42)
    out = []
    for n in [1, 2, 3, 5, 33, 64, 100, 257, 600]:
        out.append((f"rand{n}", rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))))
    n = 50
    out.append(("toeplitz", np.full(n, 0.3), np.full(n - 1, -1.7)))
    n = 60
    out.append(("clement", np.zeros(n), np.sqrt(np.arange(1, n) * (n - np.arange(1, n)))))
    n = 21
    out.append(("wilkinson21", np.abs(np.arange(n) - 10.0), np.ones(n - 1)))
    n = 40
    out.append(("diagonal", rng.standard_normal(n), np.zeros(n - 1)))
    n = 64
    out.append(("glued", np.ones(n), np.concatenate([np.full(31, 1e-9), [0.5], np.full(31, 1e-9)])))
    n = 45
    out.append(("zero", np.zeros(n), np.zeros(n - 1)))
    return out


@pytest.mark.parametrize("name,d,e", stedc_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_stedc_matches_oracle(name, d, e):
    n = len(d)
    nk = 2
    ds = np.stack([d, 2.0 * d])
    es = np.stack([e, 2.0 * e]) if n > 1 else np.zeros((nk, 0))
    w, Z, st = gpu_stedc(ds, es.reshape(nk, max(n - 1, 0)))
    assert np.all(st == 0)
    for q in range(nk):
        T = tri(ds[q], es[q]) if n > 1 else np.diag(ds[q])
        w0, Z0 = O.tridiag_ql(ds[q], es[q])
        nt = max(np.abs(T).max(), 1e-300)
        assert np.all(np.diff(w[q]) >= 0)
        assert mx(w[q] - w0) <= 16 * n * EPS * nt, f"w: {mx(w[q] - w0)}"
        assert np.linalg.norm(T @ Z[q] - Z[q] * w[q]) <= 16 * n * EPS * max(np.linalg.norm(T), 1e-300) + 1e-300
        assert mx(Z[q].T @ Z[q] - np.eye(n)) <= 16 * n * EPS, f"orth: {mx(Z[q].T @ Z[q] - np.eye(n))}"
        # vectors of well-separated eigenvalues agree with QL's up to sign
        gaps = np.minimum(np.r_[np.inf, np.diff(w0)], np.r_[np.diff(w0), np.inf]) / nt
        sep = gaps >= 1e-6
        if sep.any():
            ov = np.abs(np.sum(Z[q] * Z0, axis=0))
            assert np.max(1 - ov[sep]) <= 1e-10


@pytest.mark.parametrize("n", [2, 40, 130])
def test_back_transform_matches_oracle(n):
    kg = K()
    rng = np.random.default_rng(900 + n)
    nk = 2
    As = np.stack([rand_herm(rng, n) for _ in range(nk)])
    d, e, tau, V = gpu_hetrd(As)
    Zs = np.stack([np.linalg.qr(rng.standard_normal((n, n)))[0] for _ in range(nk)]).astype(complex)
    dV = dev(V)
    dtau = torch.from_numpy(tau).to(DEV)
    dU = dev(Zs)
    with kg.Context(0) as ctx:
        check(kg.unmtr_device(ctx, dV, dtau, n, nk, dU, n), "unmtr")
        torch.cuda.synchronize()
    U = host(dU)
    for q in range(nk):
        ref = O.apply_q(V[q], tau[q, : n - 1], Zs[q])
        assert np.abs(U[q] - ref).max() <= 32 * n * EPS


@pytest.mark.parametrize("n", [1, 3, 70, 193])
def test_eigen_hh_matches_oracle(n):
    kg = K()
    rng = np.random.default_rng(300 + n)
    nk = 3
    As = np.stack([rand_herm(rng, n) for _ in range(nk)])
    dA = dev(As)
    dw = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    dY = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    st = torch.full((nk,), -7, dtype=torch.int32, device=DEV)
    with kg.Context(0) as ctx:
        check(kg.eigh_device(ctx, dA, n, n, nk, dw, dY, st), "eigh")
        torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    w = dw.cpu().numpy()
    Y = host(dY)
    for q in range(nk):
        A = As[q]
        w0, Y0 = O.eigen_hh(A)
        nf = np.linalg.norm(A)
        assert np.abs(w[q] - w0).max() <= 1e-10 * max(np.abs(w0).max(), 1e-300)
        assert np.linalg.norm(A @ Y[q] - Y[q] * w[q]) <= 32 * n * EPS * nf
        assert np.abs(Y[q].conj().T @ Y[q] - np.eye(n)).max() <= 32 * n * EPS


def gpu_stebz(ds, es):
    kg = K()
    nk, n = ds.shape
    dd = torch.from_numpy(np.ascontiguousarray(ds)).to(DEV)
    de = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    de[:, : n - 1] = torch.from_numpy(np.ascontiguousarray(es)).to(DEV)
    dw = torch.full((nk, n), np.nan, dtype=torch.float64, device=DEV)
    with kg.Context(0) as ctx:
        check(kg.stebz_device(ctx, dd, de, n, nk, dw), "stebz")
        torch.cuda.synchronize()
    return dw.cpu().numpy()


@pytest.mark.parametrize("name,d,e", stedc_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_stebz_matches_oracle(name, d, e):
    # eigenvalues only by bisection: against the oracle's QL and its Sturm
    # bisection, within the backward-stable bound of a few eps ||T|| per value
    n = len(d)
    nk = 2
    ds = np.stack([d, -3.0 * d])
    es = np.stack([e, 3.0 * e]) if n > 1 else np.zeros((nk, 0))
    w = gpu_stebz(ds, es.reshape(nk, max(n - 1, 0)))
    for q in range(nk):
        T = tri(ds[q], es[q]) if n > 1 else np.diag(ds[q])
        nt = max(np.abs(T).max(), 1e-300)
        w0, _ = O.tridiag_ql(ds[q], es[q])
        wb = O.bisect_eigs(ds[q], es[q])
        assert np.all(np.diff(w[q]) >= 0)
        # bisection's bound has an absolute term from the pivot floor (the
        # smallest normal number), which is all there is for T = 0
        tol = 8 * n * EPS * nt + 4 * np.finfo(np.float64).tiny
        assert mx(w[q] - w0) <= tol, f"vs QL: {mx(w[q] - w0)}"
        assert mx(w[q] - wb) <= tol, f"vs bisection: {mx(w[q] - wb)}"


def test_stebz_closed_forms():
    # Toeplitz: a + 2 b cos(j pi / (n + 1)); Clement: -(n-1), -(n-3), ..., n-1
    n = 200
    a, b = 0.3, -1.7
    j = np.arange(1, n + 1)
    toe = np.sort(a + 2 * b * np.cos(j * np.pi / (n + 1)))
    m = 151
    cle = np.arange(-(m - 1), m, 2, dtype=float)
    w1 = gpu_stebz(np.full((1, n), a), np.full((1, n - 1), b))[0]
    w2 = gpu_stebz(np.zeros((1, m)), np.sqrt(np.arange(1, m) * (m - np.arange(1, m)))[None])[0]
    assert mx(w1 - toe) <= 8 * EPS * 2 * abs(b) * 4
    assert mx(w2 - cle) <= 16 * EPS * m
