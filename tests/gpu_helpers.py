"""Helpers shared by the GPU tests: device buffers in the library's
column-major layout and the phase-invariant comparison measures."""
import numpy as np
import torch

DEV = torch.device("cuda:0")
EPS = np.finfo(np.float64).eps


def K():
    from paper_1402_4247_amd import kgev
    return kgev


def dev(Ms):
    """numpy stack (nk, n, n) of mathematical matrices -> cuda column-major buffer."""
    Ms = np.asarray(Ms)
    return torch.from_numpy(np.ascontiguousarray(np.swapaxes(Ms, -1, -2))).to(DEV)


def host(t):
    """cuda column-major buffer (nk, n, n) -> numpy stack of mathematical matrices."""
    return np.swapaxes(t.detach().cpu().numpy(), -1, -2)


def zeros_c(nk, n, m=None):
    return torch.zeros((nk, m if m is not None else n, n), dtype=torch.complex128, device=DEV)


def check(st, what="call"):
    assert st == 0, f"{what} returned status {st}"


def residuals(H, S, w, C):
    r_res = np.linalg.norm(H @ C - S @ C * w) / np.linalg.norm(H)
    r_orth = np.abs(C.conj().T @ S @ C - np.eye(len(w))).max()
    return r_res, r_orth


def vec_mismatch(Ca, Cb, S, w, gap=1e-6):
    """max over non-degenerate eigenvalues of 1 - |c_a^H S c_b| (phase-invariant)."""
    n = len(w)
    scale = max(np.abs(w).max(), 1e-300)
    ok = np.ones(n, dtype=bool)
    dw = np.diff(w) / scale
    ok[:-1] &= dw >= gap
    ok[1:] &= dw >= gap
    if not ok.any():
        return 0.0
    ov = np.abs(np.einsum("ij,ij->j", Ca.conj(), S @ Cb))
    return float(np.max(1.0 - ov[ok]))
