"""GPU complex matrix product (the ZGEMMs of Parts 3-4) against the oracle's
plain triple loop, element by element, on ragged sizes spanning several
tiles.  Bound: |fl(AB) - AB| <= c k eps (|A||B|) entrywise."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, EPS, K, check

pytestmark = pytest.mark.gpu


def rnd(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("C", "N"), ("N", "C"), ("C", "C")])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (67, 45, 33), (130, 70, 129), (64, 64, 16)])
def test_zgemm_matches_triple_loop(ta, tb, m, n, k):
    kg = K()
    rng = np.random.default_rng(m * 1000 + n * 10 + k)
    batch = 3
    A = [rnd(rng, m, k) if ta == "N" else rnd(rng, k, m) for _ in range(batch)]
    B = [rnd(rng, k, n) if tb == "N" else rnd(rng, n, k) for _ in range(batch)]
    C0 = [rnd(rng, m, n) for _ in range(batch)]
    alpha, beta = 0.75 - 0.5j, -0.25 + 1j
    to = lambda Ms: torch.from_numpy(np.ascontiguousarray(np.swapaxes(np.array(Ms), -1, -2))).to(DEV)
    dA, dB, dC = to(A), to(B), to(C0)
    lda, ldb = A[0].shape[0], B[0].shape[0]
    with kg.Context(0) as ctx:
        check(kg.zgemm_device(ctx, ta, tb, m, n, k, alpha, dA, lda, A[0].size, dB, ldb, B[0].size, beta,
                              dC, m, m * n, batch))
        torch.cuda.synchronize()
    got = np.swapaxes(dC.cpu().numpy(), -1, -2)
    for q in range(batch):
        ref = O.zgemm(ta, tb, A[q], B[q], alpha=alpha, beta=beta, C=C0[q])
        opA = A[q] if ta == "N" else A[q].conj().T
        opB = B[q] if tb == "N" else B[q].conj().T
        bound = 8 * k * EPS * (abs(alpha) * np.abs(opA) @ np.abs(opB) + abs(beta) * np.abs(C0[q])) + 1e-300
        assert np.all(np.abs(got[q] - ref) <= bound), f"batch {q}: max err {np.abs(got[q]-ref).max()}"


def test_zgemm_lower_only_writes_lower():
    kg = K()
    rng = np.random.default_rng(5)
    n, k = 97, 40
    X = rnd(rng, k, n)
    G = rnd(rng, k, n)
    sentinel = 123.0 + 456.0j
    dX = torch.from_numpy(np.ascontiguousarray(X.T)).to(DEV)
    dG = torch.from_numpy(np.ascontiguousarray(G.T)).to(DEV)
    dC = torch.full((n, n), sentinel, dtype=torch.complex128, device=DEV)
    with kg.Context(0) as ctx:
        check(kg.zgemm_device(ctx, "C", "N", n, n, k, 1.0, dX, k, 0, dG, k, 0, 0.0, dC, n, 0, 1, lower=True))
        torch.cuda.synchronize()
    got = dC.cpu().numpy().T
    ref = X.conj().T @ G
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.abs(got[low] - ref[low]).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(got[~low] == sentinel)


def test_zgemm_beta_zero_ignores_nan_in_c():
    kg = K()
    rng = np.random.default_rng(6)
    A = rnd(rng, 20, 20)
    dA = torch.from_numpy(np.ascontiguousarray(A.T)).to(DEV)
    dC = torch.full((20, 20), float("nan"), dtype=torch.complex128, device=DEV)
    with kg.Context(0) as ctx:
        check(kg.zgemm_device(ctx, "N", "N", 20, 20, 20, 1.0, dA, 20, 0, dA, 20, 0, 0.0, dC, 20, 0, 1))
        torch.cuda.synchronize()
    assert np.allclose(dC.cpu().numpy().T, A @ A, atol=1e-12)
