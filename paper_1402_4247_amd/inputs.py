"""Seeded synthetic inputs for the per-k generalized eigensolve.

This module holds input generators only (no step of the eigensolve): both the
GPU tests and the CPU oracle tests draw their matrices from here.

The paper's workload is OpenMX's magnetite cell (56 atoms: 24 Fe, 32 O; 64
k-points; 1040 basis functions; Section III of arXiv:1402.4247).  Its atomic
coordinates, basis and Hamiltonian are not available, so these generators
build stand-ins with the same shapes and structure:

* ``config1``  - n = 128 dense pencil: S = I + 0.05 (A + A^H)/2 with
  A_ij = (x + iy)/sqrt(2n), x, y ~ N(0, 1); H = Q diag(lambda) Q^H with
  lambda ~ U[-1, 1] and Q Haar-distributed (QR of a complex Gaussian matrix
  with the phases of R's diagonal folded back in, Mezzadri 2007).
* ``lcao_system`` / ``lcao_hs`` - magnetite-like LCAO pencil: 56 pseudo-atoms
  (24 "Fe", 32 "O") at seeded positions in a cubic cell a = 8.4 Angstrom with
  minimum-image separation >= 1.8 Angstrom, n orbitals spread over the atoms
  as evenly as possible (Fe first for the remainder).  For orbitals i, j:
  r_ij and R_ij are the minimum-image distance and lattice vector;
  W_ij = exp(-r^2/4) u_ij e^{i k.R_ij} for orbitals on different atoms (0 on
  the same atom), S = I + c W with c = 0.5 / rho_upper(|W|), an upper
  bound on the spectral radius of the entrywise modulus (so the spectrum of
  S lies in [0.5, 1.5] for every k);
  H_ij = -exp(-r^2/3) v_ij e^{i k.R_ij} (i != j), H_ii ~ U[-0.5, 0.5].
  u, v are seeded unit-modulus phases with u_ji = conj(u_ij).
  With ``overlap="spectral"`` c = 0.5 / max_k ||W(k)||_2 over the 4x4x4
  grid instead (the bound is met at the worst k-point, so the overlaps are
  less well conditioned: lambda(S) reaches 0.5 or 1.5).
* ``known_spectrum_pencil`` - prescribed overlap condition number and known
  generalized eigenvalues: S = U diag(s) U^H, s log-spaced in [1/kappa, 1],
  H = B Q diag(lambda) Q^H B^H with B = U diag(s)^(1/2), so H c = lambda S c
  for the columns of C = U diag(s)^(-1/2) Q.
* ``lcao_near_dependent`` - one k-point of the LCAO pencil with the overlap
  scaled towards linear dependence: S = I + c W(k) with c set so that the
  smallest eigenvalue of S is delta (kappa(S) about 2 / delta).
* k-points: a 4x4x4 Monkhorst-Pack grid k = ((2p-5)/8, (2q-5)/8, (2r-5)/8)
  2 pi / a, and a 2x2x2 grid (+-1/4) 2 pi / a.

All matrices are returned as numpy arrays holding the mathematical matrix
(``M[..., i, j]`` is element (i, j)).  ``colmajor`` converts a stack to the
column-major memory layout the C ABI reads.
"""
from __future__ import annotations

import math

import numpy as np

CELL_A = 8.4          # Angstrom, cubic cell
N_FE, N_O = 24, 32    # magnetite cell composition (Section III)
MIN_SEP = 1.8         # Angstrom


def colmajor(M):
    """Stack of matrices (..., n, n) -> contiguous array whose memory holds
    each matrix column-major (element (i, j) at offset i + j*n)."""
    M = np.asarray(M)
    return np.ascontiguousarray(np.swapaxes(M, -1, -2))


def from_colmajor(buf, n, nk=None):
    """Inverse of ``colmajor`` for a flat or (nk, n, n) buffer."""
    b = np.asarray(buf)
    if nk is None:
        return np.swapaxes(b.reshape(n, n), -1, -2)
    return np.swapaxes(b.reshape(nk, n, n), -1, -2)


def haar_unitary(rng, n):
    """Haar-distributed n x n unitary (Mezzadri 2007)."""
    Z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    ph = np.diagonal(R) / np.abs(np.diagonal(R))
    return Q * ph[None, :]


def config1(n: int = 128, seed: int = 1001):
    """Dense well-conditioned pencil (H, S), both Hermitian, S SPD."""
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(2.0 * n)
    S = np.eye(n, dtype=np.complex128) + 0.05 * (A + A.conj().T) / 2.0
    lam = rng.uniform(-1.0, 1.0, n)
    Q = haar_unitary(rng, n)
    H = (Q * lam[None, :]) @ Q.conj().T
    H = (H + H.conj().T) / 2.0
    return H, S


def config1_batch(n: int, nk: int, seed: int):
    """nk independent config-1 pencils (seed, seed+1, ...), shape (nk, n, n)."""
    Hs = np.empty((nk, n, n), dtype=np.complex128)
    Ss = np.empty((nk, n, n), dtype=np.complex128)
    for k in range(nk):
        Hs[k], Ss[k] = config1(n, seed + k)
    return Hs, Ss


def mp_grid(m: int):
    """Monkhorst-Pack grid of m^3 points in units of 2 pi / a."""
    g = [(2 * p - m - 1) / (2.0 * m) for p in range(1, m + 1)]
    return np.array([(x, y, z) for x in g for y in g for z in g])


class LcaoSystem:
    """Positions, orbital layout and seeded phases of one pseudo-crystal."""

    def __init__(self, n: int, seed: int, overlap: str = "cw"):
        if overlap not in ("cw", "spectral"):
            raise ValueError(f"overlap must be 'cw' or 'spectral', not {overlap!r}")
        rng = np.random.default_rng(seed)
        natom = N_FE + N_O
        pos = []
        tries = 0
        while len(pos) < natom:
            tries += 1
            if tries > 2_000_000:
                raise RuntimeError("could not place atoms")
            p = rng.uniform(0.0, CELL_A, 3)
            ok = True
            for q in pos:
                dvec = p - q
                dvec -= CELL_A * np.round(dvec / CELL_A)
                if float(dvec @ dvec) < MIN_SEP * MIN_SEP:
                    ok = False
                    break
            if ok:
                pos.append(p)
        self.pos = np.array(pos)
        base, extra = divmod(n, natom)
        counts = np.full(natom, base, dtype=np.int64)
        counts[:extra] += 1                       # Fe atoms come first
        self.counts = counts
        self.atom_of = np.repeat(np.arange(natom), counts)
        self.n = n
        # minimum-image displacement x_b + R_ab - x_a and lattice vector R_ab
        disp = self.pos[None, :, :] - self.pos[:, None, :]
        R = -CELL_A * np.round(disp / CELL_A)
        self.R_atom = R                           # R_ba = -R_ab
        dmin = disp + R
        self.r2_atom = np.einsum("abx,abx->ab", dmin, dmin)
        ph_u = rng.uniform(0.0, 2.0 * np.pi, (n, n))
        ph_v = rng.uniform(0.0, 2.0 * np.pi, (n, n))
        self.diagH = rng.uniform(-0.5, 0.5, n)
        # Hermitian phase fields: lower triangle drawn, upper = conjugate.
        low = np.tril(np.ones((n, n), dtype=bool), -1)
        pu = np.where(low, ph_u, -ph_u.T)
        pv = np.where(low, ph_v, -ph_v.T)
        self.u = np.exp(1j * pu)
        self.v = np.exp(1j * pv)
        a = self.atom_of
        self.r2 = self.r2_atom[a[:, None], a[None, :]]
        self.same_atom = a[:, None] == a[None, :]
        magW = np.where(self.same_atom, 0.0, np.exp(-self.r2 / 4.0))
        # |W(k)_ij| does not depend on k and ||W(k)||_2 <= rho(|W|).  A few
        # power steps on a positive vector x give the Collatz-Wielandt upper
        # bound rho(|W|) <= max_i (|W| x)_i / x_i, so lambda(S(k)) is inside
        # [0.5, 1.5] for every k.
        x = np.ones(n)
        if magW.max() > 0.0:
            for _ in range(60):
                y = magW @ x
                x = y / y.max()
            self.c = 0.5 / float(((magW @ x) / x).max())
        else:
            self.c = 0.5                      # a single orbital: W = 0
        if overlap == "spectral" and magW.max() > 0.0:
            # c = 0.5 / max_k ||W(k)||_2 over the 4x4x4 grid
            self.c = 0.5 / max(float(np.abs(np.linalg.eigvalsh(self.w_matrix(k))).max()) for k in mp_grid(4))

    def real_space_blocks(self):
        """The pseudo-crystal in real space, for a Bloch sum (Band_DFT_Col
        Part 1): orbital offsets per atom, the lattice vectors in units of a,
        and for every atom pair I >= J its block of H and of S at the pair's
        minimum-image lattice vector R_IJ.  The Bloch sum of these blocks
        reproduces the lower triangles of hs(k) for every k (the diagonal
        blocks are given in full and are Hermitian)."""
        natom = len(self.counts)
        off = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int32)
        Rint = np.rint(self.R_atom / CELL_A).astype(np.int64)
        keys = {}
        Rlist = []
        hb, sb = [], []
        for I in range(natom):
            for J in range(I + 1):
                key = tuple(Rint[I, J])
                if key not in keys:
                    keys[key] = len(Rlist)
                    Rlist.append(key)
                r = keys[key]
                rows = slice(off[I], off[I + 1])
                cols = slice(off[J], off[J + 1])
                r2 = self.r2[rows, cols]
                Hb = -np.exp(-r2 / 3.0) * self.v[rows, cols]
                if I == J:
                    Hb = Hb.copy()
                    np.fill_diagonal(Hb, self.diagH[rows])
                    Sb = np.eye(off[I + 1] - off[I], dtype=np.complex128)
                else:
                    Sb = self.c * np.exp(-r2 / 4.0) * self.u[rows, cols]
                hb.append((I, J, r, Hb))
                sb.append((I, J, r, Sb))
        return off, np.array(Rlist, dtype=np.float64), hb, sb

    def _bloch(self, kfrac):
        kvec = 2.0 * np.pi / CELL_A * np.asarray(kfrac, dtype=np.float64)
        a = self.atom_of
        kR_atom = self.R_atom @ kvec                 # (natom, natom), antisymmetric
        return np.exp(1j * kR_atom[a[:, None], a[None, :]])

    def w_matrix(self, kfrac):
        """W(k): the overlap's off-site part before scaling (Hermitian)."""
        W = np.where(self.same_atom, 0.0, np.exp(-self.r2 / 4.0)) * self.u * self._bloch(kfrac)
        return np.tril(W, -1) + np.tril(W, -1).conj().T

    def hs(self, kfrac):
        """(H(k), S(k)) for k = kfrac * 2 pi / a."""
        n = self.n
        bloch = self._bloch(kfrac)
        W = np.where(self.same_atom, 0.0, np.exp(-self.r2 / 4.0)) * self.u * bloch
        S = np.eye(n, dtype=np.complex128) + self.c * W
        H = -np.exp(-self.r2 / 3.0) * self.v * bloch
        np.fill_diagonal(H, self.diagH)
        # exact Hermitian symmetry (the lower triangle is what the solver reads)
        H = np.tril(H, -1) + np.tril(H, -1).conj().T + np.diag(np.real(np.diagonal(H)))
        S = np.tril(S, -1) + np.tril(S, -1).conj().T + np.diag(np.real(np.diagonal(S)))
        return H, S


def lcao_batch(n: int, kfracs, seed: int, overlap: str = "cw"):
    """Stack (nk, n, n) of H(k), S(k) for one pseudo-crystal."""
    sysm = LcaoSystem(n, seed, overlap)
    kf = np.atleast_2d(np.asarray(kfracs, dtype=np.float64))
    Hs = np.empty((len(kf), n, n), dtype=np.complex128)
    Ss = np.empty((len(kf), n, n), dtype=np.complex128)
    for q, k in enumerate(kf):
        Hs[q], Ss[q] = sysm.hs(k)
    return Hs, Ss


def config2(n: int = 2000, nk: int = 1, seed: int = 2002):
    """Magnetite-like LCAO system; the first nk points of the 4x4x4 grid."""
    return lcao_batch(n, mp_grid(4)[:nk], seed)


def config3(n: int = 1024, nk: int = 64, seed: int = 3003):
    """All (or the first nk) k-points of the 4x4x4 grid, n = 1024."""
    return lcao_batch(n, mp_grid(4)[:nk], seed)


def config4(n: int = 4096, nk: int = 8, seed: int = 4004):
    """The 2x2x2 grid (+-1/4) 2 pi / a, n = 4096."""
    return lcao_batch(n, mp_grid(2)[:nk], seed)


def known_spectrum_pencil(n: int, kappa: float, seed: int):
    """(H, S, lam, C): S = U diag(s) U^H with s log-spaced in [1/kappa, 1] (U
    Haar, so kappa(S) = kappa), B = U diag(sqrt(s)), H = B Q diag(lam) Q^H B^H
    with Q Haar and lam uniform in [-1, 1], ascending.  C = U diag(s)^(-1/2) Q
    satisfies H C = S C diag(lam) and C^H S C = I, so lam are the generalized
    eigenvalues and C the eigenvectors, exact up to the rounding of the
    construction."""
    rng = np.random.default_rng(seed)
    U = haar_unitary(rng, n)
    Q = haar_unitary(rng, n)
    s = np.logspace(0.0, -math.log10(kappa), n) if n > 1 else np.ones(1)
    lam = np.sort(rng.uniform(-1.0, 1.0, n))
    B = U * np.sqrt(s)[None, :]
    BQ = B @ Q
    H = (BQ * lam[None, :]) @ BQ.conj().T
    S = (U * s[None, :]) @ U.conj().T
    H = (H + H.conj().T) / 2.0
    S = (S + S.conj().T) / 2.0
    C = (U / np.sqrt(s)[None, :]) @ Q
    return H, S, lam, C


def lcao_near_dependent(n: int, delta: float, seed: int, kfrac=None):
    """(H, S) of one LCAO k-point (the first 4x4x4 point by default) with
    S = I + c W(k) and c = (1 - delta) / |lambda_min(W(k))|, so that the
    smallest eigenvalue of S is delta: an overlap close to linear
    dependence, as an over-complete atomic basis gives."""
    sysm = LcaoSystem(n, seed)
    k = mp_grid(4)[0] if kfrac is None else kfrac
    W = sysm.w_matrix(k)
    lmin = float(np.linalg.eigvalsh(W)[0])
    sysm.c = (1.0 - delta) / abs(lmin)
    return sysm.hs(k)


def request_stream(count: int, seed: int = 5005, n_lo: int = 256, n_hi: int = 6000,
                   nk_max: int = 16):
    """Serving workload: list of (n, nk, seed) with n log-uniform in
    [n_lo, n_hi] and nk uniform in 1..nk_max (inputs from ``config1``)."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        nk = int(rng.integers(1, nk_max + 1))
        out.append((n, nk, seed * 1000 + q))
    return out
