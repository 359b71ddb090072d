"""Mixed-precision form (complex64 tridiagonalisation and back-transformation
of Part 4 on FP32 MFMA, FP64 tridiagonal solve, FP64 Ogita-Aishima
refinement) against the FP64 oracle, to the same bar as the FP64 path:
eigenvalues within 1e-10 relative, residual and S-orthonormality <= 1e-12."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, K, check, dev, host, residuals, vec_mismatch
from paper_1402_4247_amd import inputs as G

pytestmark = pytest.mark.gpu


def solve(Hs, Ss, iters=0, vectors=True, precision=1):
    kg = K()
    nk, n = Hs.shape[0], Hs.shape[1]
    dH, dS = dev(Hs), dev(Ss)
    dw = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    dC = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV) if vectors else None
    st = torch.full((nk,), -7, dtype=torch.int32, device=DEV)
    with kg.Context(0) as ctx:
        o = kg.make_opts(precision=precision, want_vectors=vectors, refine_iters=iters)
        check(kg.solve_k_device(ctx, dH, dS, n, n, nk, dw, dC, n, d_status=st, opts=o), "solve mixed")
        torch.cuda.synchronize()
    return dw.cpu().numpy(), (host(dC) if vectors else None), st.cpu().numpy()


@pytest.mark.parametrize("gen,n,nk", [("config1", 128, 2), ("lcao", 300, 2), ("config1", 65, 3), ("lcao", 1, 1)])
def test_mixed_matches_oracle(gen, n, nk):
    if gen == "config1":
        Hs, Ss = G.config1_batch(n, nk, 1001)
    else:
        Hs, Ss = G.config2(n, nk, 2002)
    w, C, st = solve(Hs, Ss)
    assert np.all(st == 0)
    for q in range(nk):
        s0, w0, C0 = O.solve_k(Hs[q], Ss[q])
        assert np.abs(w[q] - w0).max() <= 1e-10 * np.abs(w0).max()
        r_res, r_orth = residuals(Hs[q], Ss[q], w[q], C[q])
        assert r_res <= 1e-12 and r_orth <= 1e-12, (r_res, r_orth)
        assert vec_mismatch(C0, C[q], Ss[q], w0) <= 1e-10


def test_refinement_sweeps_reduce_the_residual():
    Hs, Ss = G.config2(200, 1, 2002)
    res, orth, sts = [], [], []
    for it in (1, 2, 3):
        w, C, st = solve(Hs, Ss, iters=it)
        r_res, r_orth = residuals(Hs[0], Ss[0], w[0], C[0])
        res.append(r_res)
        orth.append(r_orth)
        sts.append(int(st[0]))
    # one sweep from FP32 vectors is not enough, three reach FP64 accuracy;
    # the final check flags refined vectors that are visibly non-orthogonal
    # (max |Y^H Y - I| > 1e-11, which C^H S C - I reproduces to rounding)
    assert res[0] > res[2] and res[2] <= 1e-12
    assert sts[2] == 0
    for o, s_ in zip(orth, sts):
        if o > 2e-11:
            assert s_ == 2, (orth, sts)
        elif o < 5e-12:
            assert s_ == 0, (orth, sts)


def test_mixed_eigenvalues_only():
    Hs, Ss = G.config1_batch(96, 2, 77)
    w, _, st = solve(Hs, Ss, vectors=False)
    assert np.all(st == 0)
    for q in range(2):
        _, w0, _ = O.solve_k(Hs[q], Ss[q], vectors=False)
        assert np.abs(w[q] - w0).max() <= 1e-10 * np.abs(w0).max()


def cluster_pencil(n, seed):
    """Known-spectrum pencil (S = B B^H well conditioned, H = B Q diag(lam)
    Q^H B^H) whose eigenvalues include near-degenerate pairs at relative
    gaps 1e-10, 1e-8 and 1e-5 and an exactly threefold eigenvalue."""
    rng = np.random.default_rng(seed)
    base = np.sort(rng.uniform(-1.0, 1.0, n - 7))
    lam = np.sort(np.concatenate([base, [0.31, 0.31 + 1e-10, -0.47, -0.47 + 1e-8, 0.83, 0.83 + 1e-5,
                                         -0.123, -0.123, -0.123]])[:n])
    B = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    Q = G.haar_unitary(rng, n)
    BQ = B @ Q
    H = (BQ * lam[None, :]) @ BQ.conj().T
    S = B @ B.conj().T
    return 0.5 * (H + H.conj().T), 0.5 * (S + S.conj().T), lam


@pytest.mark.parametrize("precision", [0, 1])
def test_near_degenerate_clusters(precision):
    # clusters below the refinement's rotation threshold are where a
    # refinement that only re-orthogonalises inside a cluster would leave the
    # FP32 mixing of near-degenerate vectors in place
    n, nk = 160, 2
    trip = [cluster_pencil(n, 900 + q) for q in range(nk)]
    Hs = np.stack([t[0] for t in trip])
    Ss = np.stack([t[1] for t in trip])
    w, C, st = solve(Hs, Ss, precision=precision)
    assert np.all(st == 0)
    for q in range(nk):
        H, S, lam = trip[q]
        s0, w0, C0 = O.solve_k(H, S)
        assert s0 == 0
        assert np.abs(w[q] - lam).max() <= 1e-10 * np.abs(lam).max()
        assert np.abs(w[q] - w0).max() <= 1e-10 * np.abs(w0).max()
        r_res, r_orth = residuals(H, S, w[q], C[q])
        assert r_res <= 1e-12 and r_orth <= 1e-12, (r_res, r_orth)
        # vectors of eigenvalues separated by more than 1e-6 one by one, the
        # tighter clusters through their S-orthogonal projectors
        assert vec_mismatch(C0, C[q], S, w0, gap=1e-6) <= 1e-10
        for centre in (0.31, -0.47, -0.123):
            sel = np.abs(lam - centre) < 1e-7
            P = C[q][:, sel] @ C[q][:, sel].conj().T @ S
            P0 = C0[:, sel] @ C0[:, sel].conj().T @ S
            assert np.abs(P - P0).max() <= 1e-9, f"cluster at {centre}"
