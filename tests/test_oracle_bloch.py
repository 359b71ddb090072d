"""Pins of the oracle's Band_DFT_Col Part 1 (Bloch sum of real-space blocks):
k = 0 gives the plain sum, a single block gives the phase times the block,
k shifted by a reciprocal lattice vector gives the same result, blocks given
with their Hermitian partners give a Hermitian M(k), and the sum of the
synthetic crystal's blocks reproduces the generator's H(k), S(k)."""
import numpy as np

import oracle as O
from paper_1402_4247_amd import inputs as G


def _random_blocks(rng, off, nR):
    natom = len(off) - 1
    blocks = []
    for I in range(natom):
        for J in range(natom):
            for r in range(nR):
                if rng.uniform() < 0.5:
                    ni, nj = off[I + 1] - off[I], off[J + 1] - off[J]
                    M = rng.standard_normal((ni, nj)) + 1j * rng.standard_normal((ni, nj))
                    blocks.append((I, J, r, M))
    return blocks


def test_k0_is_plain_sum_and_single_block_phase():
    rng = np.random.default_rng(1)
    off = [0, 2, 5, 6]
    R = rng.integers(-2, 3, (4, 3)).astype(float)
    blocks = _random_blocks(rng, off, 4)
    M0 = O.bloch(off, blocks, R, [[0.0, 0.0, 0.0]])[0]
    ref = np.zeros((6, 6), dtype=complex)
    for I, J, r, M in blocks:
        ref[off[I]:off[I + 1], off[J]:off[J + 1]] += M
    assert np.abs(M0 - ref).max() < 1e-13
    one = [(1, 0, 2, blocks[0][3][:3, :2] if blocks[0][3].shape == (3, 2) else np.ones((3, 2)))]
    k = np.array([[0.125, -0.375, 0.25]])
    Mk = O.bloch(off, one, R, k)[0]
    ph = np.exp(2j * np.pi * (k[0] @ R[2]))
    assert np.abs(Mk[2:5, 0:2] - ph * one[0][3]).max() < 1e-14
    assert np.count_nonzero(Mk[np.ones((6, 6), bool) & ~np.pad(np.ones((3, 2), bool), ((2, 1), (0, 4)))]) == 0


def test_reciprocal_lattice_periodicity():
    rng = np.random.default_rng(2)
    off = [0, 3, 4, 7]
    R = rng.integers(-3, 4, (5, 3)).astype(float)
    blocks = _random_blocks(rng, off, 5)
    k = np.array([[0.1, 0.2, -0.3]])
    a = O.bloch(off, blocks, R, k)[0]
    b = O.bloch(off, blocks, R, k + np.array([[1.0, -2.0, 3.0]]))[0]
    assert np.abs(a - b).max() < 1e-11


def test_hermitian_partners_give_hermitian_matrix():
    rng = np.random.default_rng(3)
    off = [0, 2, 4, 7]
    R = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, -1], [0, -1, 1]], dtype=float)
    neg = {0: 0, 1: 2, 2: 1, 3: 4, 4: 3}
    blocks = []
    for I in range(3):
        for J in range(I + 1):
            for r in range(5):
                ni, nj = off[I + 1] - off[I], off[J + 1] - off[J]
                M = rng.standard_normal((ni, nj)) + 1j * rng.standard_normal((ni, nj))
                if I == J and r == 0:
                    M = (M + M.conj().T) / 2
                    blocks.append((I, J, r, M))
                    continue
                blocks.append((I, J, r, M))
                blocks.append((J, I, neg[r], M.conj().T))
    Mk = O.bloch(off, blocks, R, [[0.3, -0.1, 0.45]])[0]
    assert np.abs(Mk - Mk.conj().T).max() < 1e-13


def test_crystal_blocks_reproduce_generator():
    n = 130
    sysm = G.LcaoSystem(n, 77)
    off, R, hb, sb = sysm.real_space_blocks()
    kf = G.mp_grid(4)[:3]
    Hk = O.bloch(off, hb, R, kf)
    Sk = O.bloch(off, sb, R, kf)
    for q, k in enumerate(kf):
        H, S = sysm.hs(k)
        low = np.tril(np.ones((n, n), dtype=bool))
        assert np.abs((Hk[q] - H)[low]).max() < 1e-13
        assert np.abs((Sk[q] - S)[low]).max() < 1e-13
