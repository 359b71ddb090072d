"""Plain FP64 CPU oracle for the per-k generalized Hermitian eigensolve.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.

The arithmetic lives in ``kgev_oracle.c`` (plain C, ``double _Complex``,
unblocked textbook loops); this module only marshals numpy arrays through
ctypes.  Every function cites the passage of arXiv:1402.4247 (Section III,
Band_DFT_Col Parts 2-4 and Eigen_HH's four steps) that it follows.

Matrices are numpy arrays holding the mathematical matrix (``M[i, j]`` is
element (i, j)); they are handed to C in column-major order.  Hermitian
inputs are read from the lower triangle only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kgev_oracle.c")
_LIB = os.path.join(_HERE, "libkgev_oracle.so")

OK, ENOTPD, ENOCONV, ENONFINITE = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        lib.or_zhetrd.argtypes = [I, P, I, P, P, P, P]
        lib.or_sturm_count.argtypes = [I, P, P, D]
        lib.or_bisect_eigs.argtypes = [I, P, P, P]
        lib.or_tridiag_ql.argtypes = [I, P, P, P, I]
        lib.or_apply_q.argtypes = [I, P, P, I, P, I]
        lib.or_normalize_cols.argtypes = [I, I, P, I]
        lib.or_eigen_hh.argtypes = [I, P, I, P, P, P, P]
        lib.or_solve_k.argtypes = [I, P, I, P, I, D, P, P, I, P, P, P, P, P, P, P]
        lib.or_zgemm_ri.argtypes = [ctypes.c_char, ctypes.c_char, I, I, I, D, D, P, I, P, I, D, D,
                                    P, I]
        lib.or_fermi.argtypes = [I, I, P, I, P, D, D, D, P, P, I]
        lib.or_density.argtypes = [I, I, I, P, I, ctypes.c_long, P, I, P, I, P, D, P, P]
        lib.or_cholesky_inv.argtypes = [I, P, I, D, P, P]
        lib.or_bloch.argtypes = [I, P, I, P, P, P, P, P, P, I, P, P]
        lib.or_solve_k_prune.argtypes = [I, P, I, P, I, D, P, P, I, P]
        lib.or_density_entries.argtypes = [I, I, I, P, I, ctypes.c_long, P, I, P, I, P, D, I, P, P, P]
        lib.or_max_threads.restype = I
        lib.or_set_threads.argtypes = [I]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _colmajor(M, dtype=np.complex128):
    return np.asfortranarray(np.asarray(M, dtype=dtype))


def max_threads() -> int:
    return _L().or_max_threads()


def set_threads(t: int) -> None:
    _L().or_set_threads(int(t))


def zhetrd(A):
    """Householder tridiagonalisation (Section III, Procedures 1-6).

    Returns (d, e, tau, V) with T = tridiag(e, d, e) = Q^H A Q,
    Q = H_0 ... H_{n-2}, H_i = I - tau_i v_i v_i^H, v_i = V[:, i].
    """
    A = _colmajor(A).copy(order="F")
    n = A.shape[0]
    V = np.zeros((n, n), dtype=np.complex128, order="F")
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 1))
    tau = np.zeros(max(n - 1, 1), dtype=np.complex128)
    st = _L().or_zhetrd(n, _p(A), n, _p(V), _p(d), _p(e), _p(tau))
    if st != OK:
        raise RuntimeError(f"or_zhetrd status {st}")
    return d, e[: n - 1], tau[: n - 1], V


def sturm_count(d, e, x) -> int:
    """Number of eigenvalues of tridiag(e, d, e) strictly below x."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    if e.size == 0:
        e = np.zeros(1)
    return _L().or_sturm_count(d.size, _p(d), _p(e), float(x))


def bisect_eigs(d, e):
    """All eigenvalues of tridiag(e, d, e) by Sturm bisection (ascending)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    if e.size == 0:
        e = np.zeros(1)
    w = np.zeros(d.size)
    _L().or_bisect_eigs(d.size, _p(d), _p(e), _p(w))
    return w


def tridiag_ql(d, e, vectors: bool = True):
    """Implicit QL with Wilkinson shifts (the tridiagonal eigensolver step of
    Eigen_HH).  Returns (w ascending, Z) with Z None when vectors is False."""
    w = np.array(d, dtype=np.float64, copy=True)
    e = np.ascontiguousarray(e, dtype=np.float64)
    if e.size == 0:
        e = np.zeros(1)
    n = w.size
    Z = np.zeros((n, n), order="F") if vectors else None
    st = _L().or_tridiag_ql(n, _p(w), _p(e), _p(Z), n)
    if st != OK:
        raise RuntimeError(f"or_tridiag_ql status {st}")
    return w, Z


def apply_q(V, tau, U):
    """Rearrangement of eigenvectors: returns Q U with Q = H_0 ... H_{n-2}."""
    V = _colmajor(V)
    n = V.shape[0]
    U = _colmajor(U).copy(order="F")
    tau = np.ascontiguousarray(tau, dtype=np.complex128)
    if tau.size == 0:
        tau = np.zeros(1, dtype=np.complex128)
    _L().or_apply_q(n, _p(V), _p(tau), U.shape[1], _p(U), n)
    return U


def normalize_cols(U):
    """Unit 2-norm columns."""
    U = _colmajor(U).copy(order="F")
    _L().or_normalize_cols(U.shape[0], U.shape[1], _p(U), U.shape[0])
    return U


def eigen_hh(A, vectors: bool = True, stages: bool = False):
    """Eigen_HH (Section III): eigenvalues (ascending) and unit eigenvectors of
    the Hermitian matrix whose lower triangle is A."""
    A = _colmajor(A)
    n = A.shape[0]
    w = np.zeros(n)
    Y = np.zeros((n, n), dtype=np.complex128, order="F") if vectors else None
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 1))
    st = _L().or_eigen_hh(n, _p(A), n, _p(w), _p(Y), _p(d), _p(e))
    if st != OK:
        raise RuntimeError(f"or_eigen_hh status {st}")
    if stages:
        return w, Y, d, e[: n - 1]
    return w, Y


def zgemm(ta, tb, A, B, alpha=1.0, beta=0.0, C=None):
    """Plain triple-loop C = alpha op(A) op(B) + beta C, op in {'N', 'C'}."""
    A = _colmajor(A)
    B = _colmajor(B)
    m = A.shape[0] if ta == "N" else A.shape[1]
    k = A.shape[1] if ta == "N" else A.shape[0]
    n = B.shape[1] if tb == "N" else B.shape[0]
    Cm = np.zeros((m, n), dtype=np.complex128, order="F") if C is None else _colmajor(C).copy(order="F")
    al, be = complex(alpha), complex(beta)
    _L().or_zgemm_ri(ta.encode(), tb.encode(), m, n, k, al.real, al.imag, _p(A), A.shape[0], _p(B),
                     B.shape[0], be.real, be.imag, _p(Cm), max(m, 1))
    return Cm


def solve_k(H, S, vectors: bool = True, s_tol: float = 1e-12, stages: bool = False):
    """Band_DFT_Col Parts 2-4 for one k-point (Section III).

    Returns (status, w, C) or, with stages=True, (status, w, C, stage_dict)
    where stage_dict holds dS, eS, s, X, A, dA, eA.
    """
    H = _colmajor(H)
    S = _colmajor(S)
    n = H.shape[0]
    w = np.zeros(n)
    C = np.zeros((n, n), dtype=np.complex128, order="F") if vectors else None
    if stages:
        st_arr = dict(dS=np.zeros(n), eS=np.zeros(max(n - 1, 1)), s=np.zeros(n),
                      X=np.zeros((n, n), dtype=np.complex128, order="F"),
                      A=np.zeros((n, n), dtype=np.complex128, order="F"),
                      dA=np.zeros(n), eA=np.zeros(max(n - 1, 1)))
    else:
        st_arr = dict(dS=None, eS=None, s=None, X=None, A=None, dA=None, eA=None)
    st = _L().or_solve_k(n, _p(H), n, _p(S), n, float(s_tol), _p(w), _p(C), n,
                         _p(st_arr["dS"]), _p(st_arr["eS"]), _p(st_arr["s"]), _p(st_arr["X"]),
                         _p(st_arr["A"]), _p(st_arr["dA"]), _p(st_arr["eA"]))
    if stages:
        st_arr["eS"] = st_arr["eS"][: n - 1]
        st_arr["eA"] = st_arr["eA"][: n - 1]
        return st, w, C, st_arr
    return st, w, C


def fermi(w, wk, nelec: float, kT: float, g: float = 2.0):
    """Band_DFT_Col Part 5: chemical potential and band energy.

    ``w`` is (nk, n) eigenvalues, ``wk`` the k-point weights, ``g`` the
    electrons one state holds.  Occupations are Fermi-Dirac at temperature
    ``kT``; mu is found by bisection on the electron count.  Returns
    (mu, e_band, n_count, occ) with occ (nk, n) the unweighted occupations.
    """
    w = np.ascontiguousarray(np.atleast_2d(np.asarray(w, dtype=np.float64)))
    nk, n = w.shape
    wk = np.ascontiguousarray(np.asarray(wk, dtype=np.float64).reshape(nk))
    out = np.zeros(3)
    occ = np.zeros((nk, n))
    st = _L().or_fermi(nk, n, _p(w), n, _p(wk), float(nelec), float(kT), float(g), _p(out), _p(occ), n)
    if st != 0:
        raise ValueError("or_fermi: invalid arguments")
    return float(out[0]), float(out[1]), float(out[2]), occ


def density(C, w, occ, wk, g: float = 2.0, nocc=None, edm: bool = True):
    """Band_DFT_Col Part 6: charge density matrix and energy density matrix,
    rho = g sum_k wk_k sum_j f_kj c_kj c_kj^H and the same with weights
    f_kj lambda_kj, over the first ``nocc`` columns of each C_k.

    ``C`` is (nk, n, n) with C[k] the mathematical eigenvector matrix of
    k-point k (column j = eigenvector j).  Returns (rho, edm or None).
    """
    C = np.asarray(C, dtype=np.complex128)
    nk, n, _ = C.shape
    nocc = n if nocc is None else int(nocc)
    Cc = np.ascontiguousarray(np.transpose(C, (0, 2, 1)))      # column-major per k
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(nk, n))
    occ = np.ascontiguousarray(np.asarray(occ, dtype=np.float64).reshape(nk, n))
    wk = np.ascontiguousarray(np.asarray(wk, dtype=np.float64).reshape(nk))
    rho = np.zeros((n, n), dtype=np.complex128, order="F")
    E = np.zeros((n, n), dtype=np.complex128, order="F") if edm else None
    _L().or_density(nk, n, nocc, _p(Cc), n, n * n, _p(w), n, _p(occ), n, _p(wk), float(g), _p(rho), _p(E))
    return rho, E


def density_entries(Ccol, w, occ, wk, g, pairs, nocc=None):
    """Part 6 at the listed (a, b) entries.  ``Ccol`` is (nk, n, n) holding
    each C_k in column-major order (Ccol[k, j, i] = C_k[i, j]), as the device
    layout is.  Returns (rho_entries, edm_entries)."""
    Ccol = np.ascontiguousarray(np.asarray(Ccol, dtype=np.complex128))
    nk, n, _ = Ccol.shape
    nocc = n if nocc is None else int(nocc)
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(nk, n))
    occ = np.ascontiguousarray(np.asarray(occ, dtype=np.float64).reshape(nk, n))
    wk = np.ascontiguousarray(np.asarray(wk, dtype=np.float64).reshape(nk))
    ab = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    r = np.zeros(len(ab), dtype=np.complex128)
    e = np.zeros(len(ab), dtype=np.complex128)
    _L().or_density_entries(nk, n, nocc, _p(Ccol), n, n * n, _p(w), n, _p(occ), n, _p(wk), float(g), len(ab),
                            _p(ab), _p(r), _p(e))
    return r, e


def cholesky_inv(S, s_tol: float = 1e-12):
    """Part 2 variant (not the paper's method): S = L L^H (textbook Cholesky,
    lower triangle read) and L^{-1} by forward substitution.  Returns
    (status, L, Linv)."""
    S = _colmajor(S)
    n = S.shape[0]
    L = np.zeros((n, n), dtype=np.complex128, order="F")
    Li = np.zeros((n, n), dtype=np.complex128, order="F")
    st = _L().or_cholesky_inv(n, _p(S), n, float(s_tol), _p(L), _p(Li))
    return st, L, Li


def solve_k_prune(H, S, s_tol: float = 1e-12, vectors: bool = True):
    """Part 2 variant (not the paper's method): canonical orthogonalisation
    with pruning of the directions with s_j <= s_tol s_max, then Parts 3-4 on
    the reduced pencil.  Returns (status, nkeep, w, C) with w[nkeep:] = +inf
    and the corresponding columns of C zero."""
    H = _colmajor(H)
    S = _colmajor(S)
    n = H.shape[0]
    w = np.zeros(n)
    C = np.zeros((n, n), dtype=np.complex128, order="F") if vectors else None
    nk = ctypes.c_int(0)
    st = _L().or_solve_k_prune(n, _p(H), n, _p(S), n, float(s_tol), _p(w), _p(C), n, ctypes.byref(nk))
    return st, nk.value, w, C


def bloch(off, blocks, R, kf):
    """Band_DFT_Col Part 1: M(k) = sum over blocks (I, J, r, M_IJ) of
    exp(2 pi i k.R[r]) M_IJ placed at rows off[I].., columns off[J]..
    (fractional coordinates).  Returns (nk, n, n) mathematical matrices."""
    off = np.ascontiguousarray(np.asarray(off, dtype=np.int32))
    natom = len(off) - 1
    n = int(off[-1])
    bi = np.ascontiguousarray([b[0] for b in blocks], dtype=np.int32)
    bj = np.ascontiguousarray([b[1] for b in blocks], dtype=np.int32)
    rid = np.ascontiguousarray([b[2] for b in blocks], dtype=np.int32)
    sizes = [np.asarray(b[3]).size for b in blocks]
    doff = np.ascontiguousarray(np.concatenate([[0], np.cumsum(sizes)[:-1]]) if blocks else np.zeros(0),
                                dtype=np.int64)
    data = np.ascontiguousarray(np.concatenate([np.asfortranarray(np.asarray(b[3], dtype=np.complex128)).ravel(order="F")
                                                for b in blocks]) if blocks else np.zeros(1, dtype=np.complex128))
    R = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(-1, 3))
    kf = np.ascontiguousarray(np.asarray(kf, dtype=np.float64).reshape(-1, 3))
    nk = len(kf)
    out = np.zeros((nk, n, n), dtype=np.complex128)      # per k column-major
    _L().or_bloch(natom, _p(off), len(blocks), _p(bi), _p(bj), _p(rid), _p(doff), _p(data), _p(R), nk, _p(kf),
                  _p(out))
    return np.swapaxes(out, 1, 2).copy()
