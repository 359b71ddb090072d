"""Export and reuse of Part 2's S-orthonormaliser X (kgev_solve_k_x_device):
export gives the same results as the plain solve and an X with X^H S X = I;
reusing X for another H with the same S (the other spin), or for the vector
pass after an eigenvalues-only pass, gives bitwise the results of the plain
solve of that pencil; dS may be NULL when reusing."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, K, check, dev, host
from paper_1402_4247_amd import inputs as G

pytestmark = pytest.mark.gpu


def plain(ctx, dH, dS, n, nk, vectors=True, s_method=0):
    kg = K()
    dw = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    dC = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV) if vectors else None
    check(kg.solve_k_device(ctx, dH, dS, n, n, nk, dw, dC, n,
                            opts=kg.make_opts(want_vectors=vectors, s_method=s_method)), "solve")
    return dw, dC


def xsolve(ctx, dH, dS, n, nk, dX, mode, vectors=True, s_method=0):
    kg = K()
    dw = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    dC = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV) if vectors else None
    st = torch.full((nk,), -9, dtype=torch.int32, device=DEV)
    check(kg.solve_k_x_device(ctx, dH, dS, n, n, nk, dw, dC, n, dX, mode, d_status=st,
                              opts=kg.make_opts(want_vectors=vectors, s_method=s_method)), "x solve")
    return dw, dC, st


@pytest.mark.parametrize("s_method", [0, 1])
def test_export_then_reuse_for_the_other_spin(s_method):
    kg = K()
    n, nk = 140, 3
    Hs, Ss = G.config2(n, nk, 2002)
    H2 = Hs + np.eye(n)[None] * 0.05 + 0.01 * G.config2(n, nk, 9)[0]     # "spin-down" Hamiltonian
    dH, dS, dH2 = dev(Hs), dev(Ss), dev(H2)
    dX = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    with kg.Context(0) as ctx:
        w0, C0 = plain(ctx, dH, dS, n, nk, s_method=s_method)
        w1, C1, st1 = xsolve(ctx, dH, dS, n, nk, dX, kg.X_EXPORT, s_method=s_method)
        torch.cuda.synchronize()
        assert torch.equal(w0, w1) and torch.equal(C0, C1) and bool((st1 == 0).all())
        X = host(dX)
        for k in range(nk):
            assert np.abs(X[k].conj().T @ Ss[k] @ X[k] - np.eye(n)).max() < 1e-12
        w2r, C2r = plain(ctx, dH2, dS, n, nk, s_method=s_method)
        w2, C2, st2 = xsolve(ctx, dH2, None, n, nk, dX, kg.X_REUSE, s_method=s_method)
        torch.cuda.synchronize()
        assert torch.equal(w2, w2r) and torch.equal(C2, C2r) and bool((st2 == 0).all())


def test_eigenvalue_pass_then_vector_pass():
    kg = K()
    n, nk = 100, 2
    Hs, Ss = G.config2(n, nk, 7)
    dH, dS = dev(Hs), dev(Ss)
    dX = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    with kg.Context(0) as ctx:
        wr, Cr = plain(ctx, dH, dS, n, nk)
        w1, _, _ = xsolve(ctx, dH, dS, n, nk, dX, kg.X_EXPORT, vectors=False)
        w2, C2, _ = xsolve(ctx, dH, None, n, nk, dX, kg.X_REUSE)
        torch.cuda.synchronize()
    # the vector pass with the exported X is bitwise the plain solve; the
    # eigenvalue pass finds the eigenvalues of the same tridiagonal matrices
    # by bisection instead of divide and conquer, so it agrees to rounding
    assert torch.equal(w2, wr) and torch.equal(C2, Cr)
    wr_h, w1_h = wr.cpu().numpy(), w1.cpu().numpy()
    for k in range(nk):
        scale = np.abs(wr_h[k]).max()
        assert np.abs(w1_h[k] - wr_h[k]).max() <= 8 * n * np.finfo(np.float64).eps * scale
        s0, w0, _ = O.solve_k(Hs[k], Ss[k], vectors=False)
        assert s0 == 0 and np.abs(w1_h[k] - w0).max() <= 1e-10 * np.abs(w0).max()


def test_argument_errors():
    kg = K()
    n, nk = 16, 1
    Hs, Ss = G.config2(n, nk, 3)
    dH, dS = dev(Hs), dev(Ss)
    dX = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    dw = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    with kg.Context(0) as ctx:
        o = kg.make_opts(want_vectors=False)
        assert kg.solve_k_x_device(ctx, dH, None, n, n, nk, dw, None, n, dX, kg.X_EXPORT, opts=o) == -3
        assert kg.solve_k_x_device(ctx, dH, dS, n, n, nk, dw, None, n, None, kg.X_EXPORT, opts=o) == -10
        assert kg.solve_k_x_device(ctx, dH, dS, n, n, nk, dw, None, n, dX, 5, opts=o) == -11
        op = kg.make_opts(want_vectors=False, s_method=kg.S_PRUNE)
        assert kg.solve_k_x_device(ctx, dH, None, n, n, nk, dw, None, n, dX, kg.X_REUSE, opts=op) == -102
