"""Pruned canonical orthogonalisation (opts.s_method = KGEV_S_PRUNE) on the
GPU against the oracle's pruned form: the number of kept directions, the
kept eigenvalues (within 1e-10 max|l|), the kept eigenvectors (phase-
invariant, S-orthonormal), +inf eigenvalues and zero columns for the pruned
directions, a closed-form diagonal case, and equality with the paper's form
when nothing is pruned."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, K, check, dev, host, vec_mismatch
from paper_1402_4247_amd import inputs as G

pytestmark = pytest.mark.gpu


def solve(Hs, Ss, s_method, vectors=True):
    kg = K()
    nk, n = Hs.shape[0], Hs.shape[1]
    dH, dS = dev(Hs), dev(Ss)
    dw = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    dC = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV) if vectors else None
    st = torch.full((nk,), -7, dtype=torch.int32, device=DEV)
    with kg.Context(0) as ctx:
        o = kg.make_opts(s_method=s_method, want_vectors=vectors)
        check(kg.solve_k_device(ctx, dH, dS, n, n, nk, dw, dC, n, d_status=st, opts=o), "solve")
        torch.cuda.synchronize()
    return dw.cpu().numpy(), (host(dC) if vectors else None), st.cpu().numpy()


def rank_deficient(n, r, seed):
    rng = np.random.default_rng(seed)
    B = (rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))) / np.sqrt(2 * n)
    S = B @ B.conj().T
    S = (S + S.conj().T) / 2
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = (A + A.conj().T) / np.sqrt(8 * n)
    return H, S


def test_nothing_pruned_equals_paper_form():
    kg = K()
    Hs, Ss = G.config2(120, 2, 2002)
    w1, C1, s1 = solve(Hs, Ss, kg.S_EIG)
    w2, C2, s2 = solve(Hs, Ss, kg.S_PRUNE)
    assert np.all(s1 == 0) and np.all(s2 == 0)
    assert np.array_equal(w1, w2) and np.array_equal(C1, C2)


@pytest.mark.parametrize("n,r", [(40, 31), (150, 130), (130, 64)])
def test_rank_deficient_overlap_matches_oracle(n, r):
    kg = K()
    H, S = rank_deficient(n, r, 300 + n)
    # the paper's form rejects this S
    _, _, st_eig = solve(H[None], S[None], kg.S_EIG, vectors=False)
    assert st_eig.tolist() == [1]
    w, C, st = solve(H[None], S[None], kg.S_PRUNE)
    st0, m0, w0, C0 = O.solve_k_prune(H, S)
    assert st0 == 0 and m0 == r and st.tolist() == [0]
    w, C = w[0], C[0]
    m = int(np.isfinite(w).sum())
    assert m == m0
    assert np.all(np.isinf(w[m:])) and np.all(C[:, m:] == 0)
    assert np.abs(w[:m] - w0[:m]).max() <= 1e-10 * np.abs(w0[:m]).max()
    Ck = C[:, :m]
    assert np.abs(Ck.conj().T @ S @ Ck - np.eye(m)).max() <= 1e-10
    assert vec_mismatch(C0[:, :m], Ck, S, w0[:m]) <= 1e-8


def test_diagonal_closed_form():
    kg = K()
    h = np.array([3.0, -1.0, 2.0, 5.0, 0.5, -4.0, 1.5, 0.25])
    s = np.array([2.0, 1.0, 0.0, 4.0, 1e-20, 0.5, 3.0, 0.0])
    w, C, st = solve(np.diag(h).astype(complex)[None], np.diag(s).astype(complex)[None], kg.S_PRUNE)
    keep = s > 1e-12 * s.max()
    m = int(keep.sum())
    assert st.tolist() == [0]
    assert np.abs(w[0, :m] - np.sort(h[keep] / s[keep])).max() < 1e-14
    assert np.all(np.isinf(w[0, m:])) and np.all(C[0][:, m:] == 0)


def test_eigenvalues_only():
    kg = K()
    H, S = rank_deficient(90, 70, 9)
    w, _, st = solve(H[None], S[None], kg.S_PRUNE, vectors=False)
    st0, m0, w0, _ = O.solve_k_prune(H, S, vectors=False)
    assert st.tolist() == [0] and int(np.isfinite(w[0]).sum()) == m0
    assert np.abs(w[0, :m0] - w0[:m0]).max() <= 1e-10 * np.abs(w0[:m0]).max()
