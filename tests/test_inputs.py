"""Seeded input generators: determinism, Hermitian structure, SPD S."""
import numpy as np

from paper_1402_4247_amd import inputs as G


def test_config1_deterministic_and_spd():
    H1, S1 = G.config1(128, 1001)
    H2, S2 = G.config1(128, 1001)
    assert np.array_equal(H1, H2) and np.array_equal(S1, S2)
    assert np.array_equal(H1, H1.conj().T) and np.array_equal(S1, S1.conj().T)
    assert np.linalg.eigvalsh(S1).min() >= 0.5


def test_lcao_hermitian_spd_and_k_structure():
    Hs, Ss = G.config2(112, 3, 2002)
    for H, S in zip(Hs, Ss):
        assert np.array_equal(H, H.conj().T) and np.array_equal(S, S.conj().T)
        ev = np.linalg.eigvalsh(S)
        assert ev.min() >= 0.5 and ev.max() <= 1.5
    # k-dependence enters only through phases: |S(k)_ij| is k-independent
    assert np.allclose(np.abs(Ss[0]), np.abs(Ss[1]))
    # orbitals spread over 56 atoms
    sysm = G.LcaoSystem(2000, 2002)
    assert sysm.counts.sum() == 2000 and sysm.counts.max() - sysm.counts.min() <= 1


def test_k_grids():
    g = G.mp_grid(4)
    assert g.shape == (64, 3) and np.allclose(g[0], [-3 / 8] * 3)
    assert np.allclose(np.sort(np.unique(g)), [-3 / 8, -1 / 8, 1 / 8, 3 / 8])
    assert G.mp_grid(2).shape == (8, 3) and np.allclose(np.abs(G.mp_grid(2)), 0.25)


def test_colmajor_roundtrip():
    H, S = G.config1(9, 1)
    buf = G.colmajor(H)
    assert buf.ravel()[1] == H[1, 0]                  # element (1,0) at offset 1
    assert np.array_equal(G.from_colmajor(buf, 9), H)


def test_request_stream():
    reqs = G.request_stream(200, 5005)
    ns = np.array([r[0] for r in reqs])
    nks = np.array([r[1] for r in reqs])
    assert ns.min() >= 256 and ns.max() <= 6000 and nks.min() >= 1 and nks.max() <= 16
    assert reqs == G.request_stream(200, 5005)
