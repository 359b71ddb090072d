"""The Cholesky form of Part 2 (opts.s_method = KGEV_S_CHOLESKY, X = L^{-H} J,
J the reversal of the column order):
the same eigenpairs as the oracle's (paper's) form to the path's bar
(eigenvalues within 1e-10 max|l|, residuals <= 1e-12, eigenvectors of
non-degenerate eigenvalues equal up to phase), its definiteness status, and
its combination with the mixed-precision form."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, K, check, dev, host, residuals, vec_mismatch
from paper_1402_4247_amd import inputs as G

pytestmark = pytest.mark.gpu


def solve(Hs, Ss, precision=0, s_tol=0.0):
    kg = K()
    nk, n = Hs.shape[0], Hs.shape[1]
    dH, dS = dev(Hs), dev(Ss)
    dw = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    dC = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    st = torch.full((nk,), -7, dtype=torch.int32, device=DEV)
    with kg.Context(0) as ctx:
        o = kg.make_opts(precision=precision, s_method=kg.S_CHOLESKY, s_tol=s_tol)
        check(kg.solve_k_device(ctx, dH, dS, n, n, nk, dw, dC, n, d_status=st, opts=o), "solve")
        torch.cuda.synchronize()
    return dw.cpu().numpy(), host(dC), st.cpu().numpy()


@pytest.mark.parametrize("n,nk", [(1, 1), (2, 2), (63, 2), (64, 1), (65, 2), (150, 2), (300, 1)])
def test_cholesky_form_matches_oracle(n, nk):
    Hs, Ss = G.config2(n, nk, 2002 + n)
    w, C, st = solve(Hs, Ss)
    assert np.all(st == 0)
    for k in range(nk):
        st0, w0, C0 = O.solve_k(Hs[k], Ss[k])
        assert st0 == 0
        assert np.abs(w[k] - w0).max() <= 1e-10 * np.abs(w0).max()
        r_res, r_orth = residuals(Hs[k], Ss[k], w[k], C[k])
        assert r_res <= 1e-12 and r_orth <= 1e-12, (r_res, r_orth)
        assert vec_mismatch(C0, C[k], Ss[k], w0) <= 1e-10


def test_cholesky_form_config1():
    Hs, Ss = G.config1_batch(128, 2, 1001)
    w, C, st = solve(Hs, Ss)
    assert np.all(st == 0)
    for k in range(2):
        st0, w0, _ = O.solve_k(Hs[k], Ss[k])
        assert np.abs(w[k] - w0).max() <= 1e-10 * np.abs(w0).max()
        r_res, r_orth = residuals(Hs[k], Ss[k], w[k], C[k])
        assert r_res <= 1e-12 and r_orth <= 1e-12


def test_cholesky_form_not_positive_definite():
    Hs, Ss = G.config1_batch(70, 3, 5)
    Ss = Ss.copy()
    Ss[1] = -Ss[1]
    _, _, st = solve(Hs, Ss)
    assert st.tolist() == [0, 1, 0]


def test_cholesky_form_with_mixed_precision():
    Hs, Ss = G.config2(200, 2, 77)
    w, C, st = solve(Hs, Ss, precision=1)
    assert np.all(st == 0)
    for k in range(2):
        st0, w0, _ = O.solve_k(Hs[k], Ss[k])
        assert np.abs(w[k] - w0).max() <= 1e-10 * np.abs(w0).max()
        r_res, r_orth = residuals(Hs[k], Ss[k], w[k], C[k])
        assert r_res <= 1e-12 and r_orth <= 1e-12


@pytest.mark.parametrize("n", [63, 130])
def test_cholesky_x_matches_oracle_factor(n):
    # the exported X is the oracle's L^{-H} (textbook Cholesky and forward
    # substitution) with its columns in reverse order, entry by entry within
    # the first-order error of a triangular inverse, c n eps |L^{-1}| |L| |L^{-1}|
    kg = K()
    nk = 2
    Hs, Ss = G.config2(n, nk, 40 + n)
    dH, dS = dev(Hs), dev(Ss)
    dX = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    dw = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    st = torch.full((nk,), -9, dtype=torch.int32, device=DEV)
    with kg.Context(0) as ctx:
        o = kg.make_opts(want_vectors=False, s_method=kg.S_CHOLESKY)
        check(kg.solve_k_x_device(ctx, dH, dS, n, n, nk, dw, None, n, dX, kg.X_EXPORT, d_status=st, opts=o), "x")
        torch.cuda.synchronize()
    assert bool((st == 0).all())
    X = host(dX)
    for k in range(nk):
        s0, L, Li = O.cholesky_inv(Ss[k])
        assert s0 == 0
        Xo = Li.conj().T[:, ::-1]
        bound = 8 * n * np.finfo(np.float64).eps * (np.abs(Li) @ np.abs(L) @ np.abs(Li)).conj().T[:, ::-1]
        assert np.all(np.abs(X[k] - Xo) <= bound + 1e-300)
