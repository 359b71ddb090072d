"""Degenerate and special pencils through the whole GPU solve, against the
oracle and against what the mathematics fixes:

* H = S: every eigenvalue is 1;
* H = 0: every eigenvalue is 0 and C is any S-orthonormal basis;
* S = I: the standard Hermitian eigenproblem;
* eigenvalues of high multiplicity (H = B Q diag(l) Q^H B^H with S = B B^H,
  so the pencil's eigenvalues are exactly l): the eigenvalues, the residuals,
  S-orthonormality, and each multiple eigenvalue's eigenspace (its
  S-orthogonal projector C_l C_l^H S, which does not depend on the basis
  chosen inside it) against the oracle's;
* a long batch of odd size (37 k-points), every k against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, K, check, dev, host, residuals, vec_mismatch
from paper_1402_4247_amd import inputs as G

pytestmark = pytest.mark.gpu


def gpu_solve(Hs, Ss):
    kg = K()
    nk, n = Hs.shape[0], Hs.shape[1]
    dH, dS = dev(Hs), dev(Ss)
    dw = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    dC = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    st = torch.full((nk,), -7, dtype=torch.int32, device=DEV)
    with kg.Context(0) as ctx:
        check(kg.solve_k_device(ctx, dH, dS, n, n, nk, dw, dC, n, d_status=st), "solve_k_device")
        torch.cuda.synchronize()
    return dw.cpu().numpy(), host(dC), st.cpu().numpy()


def s_orth(C, S):
    return np.abs(C.conj().T @ S @ C - np.eye(C.shape[1])).max()


def test_h_equals_s():
    n, nk = 150, 2
    _, Ss = G.config2(n, nk, 2002)
    w, C, st = gpu_solve(Ss.copy(), Ss)
    assert np.all(st == 0)
    for q in range(nk):
        assert np.abs(w[q] - 1.0).max() <= 1e-12
        assert s_orth(C[q], Ss[q]) <= 1e-12
        assert np.linalg.norm(Ss[q] @ C[q] - Ss[q] @ C[q] * w[q]) <= 1e-12 * np.linalg.norm(Ss[q])


def test_h_zero():
    n, nk = 97, 2
    _, Ss = G.config1_batch(n, nk, 7)
    w, C, st = gpu_solve(np.zeros_like(Ss), Ss)
    assert np.all(st == 0)
    assert np.abs(w).max() <= 1e-14
    for q in range(nk):
        assert s_orth(C[q], Ss[q]) <= 1e-12


def test_identity_overlap():
    n, nk = 130, 2
    Hs, _ = G.config1_batch(n, nk, 9)
    Ss = np.broadcast_to(np.eye(n, dtype=np.complex128), (nk, n, n)).copy()
    w, C, st = gpu_solve(Hs, Ss)
    assert np.all(st == 0)
    for q in range(nk):
        s0, w0, C0 = O.solve_k(Hs[q], Ss[q])
        assert s0 == 0
        assert np.abs(w[q] - w0).max() <= 1e-10 * np.abs(w0).max()
        r_res, r_orth = residuals(Hs[q], Ss[q], w[q], C[q])
        assert r_res <= 1e-12 and r_orth <= 1e-12
        assert vec_mismatch(C0, C[q], Ss[q], w0) <= 1e-10


@pytest.mark.parametrize("n,levels", [(120, 5), (200, 3)])
def test_multiple_eigenvalues(n, levels):
    rng = np.random.default_rng(100 + n)
    nk = 2
    lam = np.sort(np.repeat(np.linspace(-1.0, 1.0, levels), n // levels + 1)[:n])
    Hs = np.empty((nk, n, n), dtype=np.complex128)
    Ss = np.empty_like(Hs)
    for q in range(nk):
        B = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
        Q, R = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        Q = Q * (np.diagonal(R) / np.abs(np.diagonal(R)))
        H = B @ Q @ np.diag(lam) @ Q.conj().T @ B.conj().T
        S = B @ B.conj().T
        Hs[q] = 0.5 * (H + H.conj().T)
        Ss[q] = 0.5 * (S + S.conj().T)
    w, C, st = gpu_solve(Hs, Ss)
    assert np.all(st == 0)
    for q in range(nk):
        s0, w0, C0 = O.solve_k(Hs[q], Ss[q])
        assert s0 == 0
        assert np.abs(w[q] - lam).max() <= 1e-10 and np.abs(w0 - lam).max() <= 1e-10
        r_res, r_orth = residuals(Hs[q], Ss[q], w[q], C[q])
        assert r_res <= 1e-12 and r_orth <= 1e-12
        for lv in np.unique(lam):
            sel = np.abs(lam - lv) < 1e-12
            P = C[q][:, sel] @ C[q][:, sel].conj().T @ Ss[q]
            P0 = C0[:, sel] @ C0[:, sel].conj().T @ Ss[q]
            assert np.abs(P - P0).max() <= 1e-9, f"eigenspace of {lv}"


def test_long_odd_batch():
    n, nk = 40, 37
    Hs, Ss = G.config1_batch(n, nk, 11)
    w, C, st = gpu_solve(Hs, Ss)
    assert np.all(st == 0)
    for q in range(nk):
        s0, w0, C0 = O.solve_k(Hs[q], Ss[q])
        assert s0 == 0
        assert np.abs(w[q] - w0).max() <= 1e-10 * np.abs(w0).max()
        r_res, r_orth = residuals(Hs[q], Ss[q], w[q], C[q])
        assert r_res <= 1e-12 and r_orth <= 1e-12
        assert vec_mismatch(C0, C[q], Ss[q], w0) <= 1e-10
