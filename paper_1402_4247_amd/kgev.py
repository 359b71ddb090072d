"""Python binding of the HIP library ``libkgev.so`` (C ABI in include/kgev.h).

Argument marshalling only: every step of the eigensolve runs in the library's
HIP kernels.  PyTorch supplies device memory and the current HIP stream.
Loading fails loudly when the library has not been built; there is no
fallback of any kind.

Matrices handed to the library are column-major.  For a stack of matrices
held as a torch tensor ``M`` of shape (nk, n, n) with ``M[q, i, j]`` the
element (i, j), ``colmajor(M)`` gives the buffer the library reads.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkgev.so")

OK, ENOTPD, ENOCONV, ENONFINITE = 0, 1, 2, 3
ENOMEM, EDEVICE, EUNSUPPORTED = -100, -101, -102
PREC_FP64, PREC_FP32_REFINE = 0, 1


class KgevError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f"{fn} failed with status {status} ({status_str(status)})")
        self.status = status


class Z(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nk", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("dH", ctypes.c_void_p), ("dS", ctypes.c_void_p), ("dw", ctypes.c_void_p),
                ("dC", ctypes.c_void_p), ("ldc", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("bad_k", ctypes.c_int64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("footprint", ctypes.c_size_t)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("want_vectors", ctypes.c_int32),
                ("panel_nb", ctypes.c_int32), ("refine_iters", ctypes.c_int32),
                ("s_tol", ctypes.c_double), ("use_graph", ctypes.c_int32), ("streams", ctypes.c_int32),
                ("s_method", ctypes.c_int32), ("hemv_slots", ctypes.c_int32), ("gemm_slots", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class Problem(ctypes.Structure):
    """kgev_problem: one system of a kgev_solve_batch_device call."""
    _fields_ = [("n", ctypes.c_int64), ("ld", ctypes.c_int64), ("nk", ctypes.c_int64),
                ("dH", ctypes.c_void_p), ("dS", ctypes.c_void_p), ("dw", ctypes.c_void_p),
                ("dC", ctypes.c_void_p), ("ldc", ctypes.c_int64), ("d_status", ctypes.c_void_p)]


EXPORTS = ["kgev_opts_default", "kgev_status_str", "kgev_create", "kgev_destroy",
           "kgev_workspace_bytes", "kgev_solve_k", "kgev_solve_k_device", "kgev_hetrd_device",
           "kgev_stedc_device", "kgev_unmtr_device", "kgev_eigh_device", "kgev_zgemm_device",
           "kgev_profile_begin", "kgev_profile_end", "kgev_server_create", "kgev_server_submit",
           "kgev_server_poll", "kgev_server_wait", "kgev_server_destroy", "kgev_server_set_bypass", "kgev_autotune",
           "kgev_fermi_device", "kgev_density_workspace_bytes", "kgev_density_device", "kgev_bloch_device",
           "kgev_solve_k_x_device", "kgev_batch_workspace_bytes", "kgev_solve_batch_device",
           "kgev_solve_k_device_noalloc", "kgev_stebz_device", "kgev_tuned_params"]
NOALLOC_SCRATCH_BYTES = 128 << 20
PHASE_HEMV, PHASE_GEMM = 1, 2
S_EIG, S_CHOLESKY, S_PRUNE = 0, 1, 2


def _load():
    # PyTorch bundles its own HIP runtime.  Load it first when it is installed,
    # so that the library binds to that same runtime (one runtime per process:
    # device pointers and streams from torch are then valid here).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1402_4247_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.kgev_opts_default.argtypes = [ctypes.POINTER(Opts)]
    lib.kgev_status_str.argtypes = [I32]
    lib.kgev_status_str.restype = ctypes.c_char_p
    lib.kgev_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
    lib.kgev_create.restype = I32
    lib.kgev_destroy.argtypes = [P]
    lib.kgev_workspace_bytes.argtypes = [I64, I64, ctypes.POINTER(Opts)]
    lib.kgev_workspace_bytes.restype = ctypes.c_size_t
    lib.kgev_solve_k.argtypes = [P, P, P, I64, I64, P, P, ctypes.POINTER(Opts), ctypes.POINTER(I64)]
    lib.kgev_solve_k.restype = I32
    lib.kgev_solve_k_device.argtypes = [P, P, P, I64, I64, I64, P, P, I64, P, ctypes.c_size_t, P,
                                        ctypes.POINTER(Opts), P]
    lib.kgev_solve_k_device.restype = I32
    lib.kgev_solve_k_device_noalloc.argtypes = [P, P, P, I64, I64, I64, P, P, I64, P, ctypes.POINTER(Opts), P]
    lib.kgev_solve_k_device_noalloc.restype = I32
    lib.kgev_hetrd_device.argtypes = [P, P, I64, I64, I64, P, P, P, P, ctypes.POINTER(Opts), P]
    lib.kgev_hetrd_device.restype = I32
    lib.kgev_stedc_device.argtypes = [P, P, P, I64, I64, P, P, P, P]
    lib.kgev_stedc_device.restype = I32
    lib.kgev_stebz_device.argtypes = [P, P, P, I64, I64, P, P]
    lib.kgev_stebz_device.restype = I32
    lib.kgev_unmtr_device.argtypes = [P, P, P, I64, I64, P, I64, P]
    lib.kgev_unmtr_device.restype = I32
    lib.kgev_eigh_device.argtypes = [P, P, I64, I64, I64, P, P, P, ctypes.POINTER(Opts), P]
    lib.kgev_eigh_device.restype = I32
    lib.kgev_fermi_device.argtypes = [P, P, I64, I64, I64, P, D, D, D, P, I64, P, P, P]
    lib.kgev_fermi_device.restype = I32
    lib.kgev_density_workspace_bytes.argtypes = [I64, I64, I64]
    lib.kgev_density_workspace_bytes.restype = ctypes.c_size_t
    lib.kgev_density_device.argtypes = [P, P, I64, I64, I64, I64, P, I64, P, I64, P, D, P, P, I64, P,
                                        ctypes.c_size_t, P]
    lib.kgev_density_device.restype = I32
    lib.kgev_bloch_device.argtypes = [P, I32, P, I64, P, P, P, P, P, I64, I64, P, I64, P, P, P]
    lib.kgev_bloch_device.restype = I32
    lib.kgev_solve_k_x_device.argtypes = [P, P, P, I64, I64, I64, P, P, I64, P, I32, P, ctypes.c_size_t, P,
                                          ctypes.POINTER(Opts), P]
    lib.kgev_solve_k_x_device.restype = I32
    lib.kgev_batch_workspace_bytes.argtypes = [ctypes.POINTER(Problem), I64, ctypes.POINTER(Opts)]
    lib.kgev_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.kgev_solve_batch_device.argtypes = [P, ctypes.POINTER(Problem), I64, P, ctypes.c_size_t,
                                            ctypes.POINTER(Opts), P]
    lib.kgev_solve_batch_device.restype = I32
    lib.kgev_zgemm_device.argtypes = [P, ctypes.c_char, ctypes.c_char, I64, I64, I64, Z, P, I64, I64,
                                      P, I64, I64, Z, P, I64, I64, I64, I32, P]
    lib.kgev_zgemm_device.restype = I32
    lib.kgev_profile_begin.argtypes = [P, I32, I32]
    lib.kgev_profile_begin.restype = I32
    lib.kgev_profile_end.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(D),
                                     ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.kgev_profile_end.restype = I32
    lib.kgev_server_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.c_size_t, I32]
    lib.kgev_server_create.restype = I32
    lib.kgev_server_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.kgev_server_submit.restype = I32
    lib.kgev_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(I32)]
    lib.kgev_server_poll.restype = I32
    lib.kgev_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result)]
    lib.kgev_server_wait.restype = I32
    lib.kgev_server_destroy.argtypes = [P]
    lib.kgev_server_set_bypass.argtypes = [P, I32]
    lib.kgev_server_set_bypass.restype = I32
    lib.kgev_autotune.argtypes = [P, I64, I32, ctypes.POINTER(I32)]
    lib.kgev_autotune.restype = I32
    lib.kgev_tuned_params.argtypes = [P, I64, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32),
                                      ctypes.POINTER(I32)]
    lib.kgev_tuned_params.restype = I32
    return lib


lib = _load()


def status_str(st: int) -> str:
    return lib.kgev_status_str(int(st)).decode()


def _check(fn, st):
    if st != OK:
        raise KgevError(fn, st)


def make_opts(precision=PREC_FP64, want_vectors=True, panel_nb=0, refine_iters=0, s_tol=0.0,
              use_graph=False, streams=0, s_method=0, hemv_slots=0, gemm_slots=0) -> Opts:
    o = Opts()
    lib.kgev_opts_default(ctypes.byref(o))
    o.hemv_slots = hemv_slots
    o.gemm_slots = gemm_slots
    o.use_graph = 1 if use_graph else 0
    o.streams = streams
    o.s_method = s_method
    o.precision = precision
    o.want_vectors = 1 if want_vectors else 0
    o.panel_nb = panel_nb
    o.refine_iters = refine_iters
    o.s_tol = s_tol
    return o


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def colmajor(M):
    """(..., n, n) torch tensor -> contiguous tensor whose memory holds each
    matrix column-major."""
    return M.transpose(-1, -2).contiguous()


def from_colmajor(buf):
    return buf.transpose(-1, -2)


class Context:
    """Owns one kgev_ctx on a HIP device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check("kgev_create", lib.kgev_create(ctypes.byref(h), int(device)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib.kgev_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def workspace_bytes(n: int, nk: int, opts: Opts | None = None) -> int:
    return int(lib.kgev_workspace_bytes(n, nk, None if opts is None else ctypes.byref(opts)))


def solve_k_device(ctx: Context, dH, dS, n, ld, nk, dw, dC, ldc, dwork=None, work_bytes=0, d_status=None,
                   opts: Opts | None = None, stream=None) -> int:
    """kgev_solve_k_device on torch device tensors (column-major buffers)."""
    return lib.kgev_solve_k_device(ctx.handle, _ptr(dH), _ptr(dS), n, ld, nk, _ptr(dw), _ptr(dC), ldc,
                                   _ptr(dwork), work_bytes, _ptr(d_status),
                                   None if opts is None else ctypes.byref(opts), _stream(stream))


def solve_k_device_noalloc(ctx: Context, dH, dS, n, ld, nk, dw, dC, ldc, d_status=None,
                           opts: Opts | None = None, stream=None) -> int:
    """kgev_solve_k_device_noalloc: the same solve with the library's static
    per-GPU workspace (no device allocation)."""
    return lib.kgev_solve_k_device_noalloc(ctx.handle, _ptr(dH), _ptr(dS), n, ld, nk, _ptr(dw), _ptr(dC), ldc,
                                           _ptr(d_status), None if opts is None else ctypes.byref(opts),
                                           _stream(stream))


X_EXPORT, X_REUSE = 0, 1


def solve_k_x_device(ctx: Context, dH, dS, n, ld, nk, dw, dC, ldc, dX, x_mode, dwork=None, work_bytes=0,
                     d_status=None, opts: Opts | None = None, stream=None) -> int:
    """kgev_solve_k_x_device: the per-k solve exporting (X_EXPORT) or reusing
    (X_REUSE) Part 2's S-orthonormaliser X."""
    return lib.kgev_solve_k_x_device(ctx.handle, _ptr(dH), _ptr(dS), n, ld, nk, _ptr(dw), _ptr(dC), ldc, _ptr(dX),
                                     int(x_mode), _ptr(dwork), work_bytes, _ptr(d_status),
                                     None if opts is None else ctypes.byref(opts), _stream(stream))


def problem(dH, dS, n, ld, nk, dw, dC=None, ldc=0, d_status=None) -> Problem:
    """One kgev_problem from device tensors (column-major per k)."""
    def addr(t):
        return None if t is None else t.data_ptr()
    return Problem(n, ld, nk, addr(dH), addr(dS), addr(dw), addr(dC), ldc, addr(d_status))


def batch_workspace_bytes(problems, opts: Opts | None = None) -> int:
    arr = (Problem * len(problems))(*problems)
    return lib.kgev_batch_workspace_bytes(arr, len(problems), None if opts is None else ctypes.byref(opts))


def solve_batch_device(ctx: Context, problems, dwork=None, work_bytes=0, opts: Opts | None = None,
                       stream=None) -> int:
    """kgev_solve_batch_device: systems of uneven order in one call."""
    arr = (Problem * len(problems))(*problems)
    return lib.kgev_solve_batch_device(ctx.handle, arr, len(problems), _ptr(dwork), work_bytes,
                                       None if opts is None else ctypes.byref(opts), _stream(stream))


def solve_k(ctx: Context, H, S, n, nk, w, C, opts: Opts | None = None):
    """kgev_solve_k on host numpy buffers (complex128, column-major per k).
    Returns (status, bad_k)."""
    bad = ctypes.c_int64(-1)
    st = lib.kgev_solve_k(ctx.handle, H.ctypes.data_as(ctypes.c_void_p), S.ctypes.data_as(ctypes.c_void_p),
                          n, nk, w.ctypes.data_as(ctypes.c_void_p),
                          None if C is None else C.ctypes.data_as(ctypes.c_void_p),
                          None if opts is None else ctypes.byref(opts), ctypes.byref(bad))
    return st, bad.value


def hetrd_device(ctx, dA, n, lda, nk, dd, de, dtau, dV, opts=None, stream=None) -> int:
    return lib.kgev_hetrd_device(ctx.handle, _ptr(dA), n, lda, nk, _ptr(dd), _ptr(de), _ptr(dtau), _ptr(dV),
                                 None if opts is None else ctypes.byref(opts), _stream(stream))


def stedc_device(ctx, dd, de, n, nk, dw, dZ, d_status=None, stream=None) -> int:
    return lib.kgev_stedc_device(ctx.handle, _ptr(dd), _ptr(de), n, nk, _ptr(dw), _ptr(dZ), _ptr(d_status),
                                 _stream(stream))


def stebz_device(ctx, dd, de, n, nk, dw, stream=None) -> int:
    """kgev_stebz_device: tridiagonal eigenvalues by bisection."""
    return lib.kgev_stebz_device(ctx.handle, _ptr(dd), _ptr(de), n, nk, _ptr(dw), _stream(stream))


def unmtr_device(ctx, dV, dtau, n, nk, dU, ldu, stream=None) -> int:
    return lib.kgev_unmtr_device(ctx.handle, _ptr(dV), _ptr(dtau), n, nk, _ptr(dU), ldu, _stream(stream))


def eigh_device(ctx, dA, n, lda, nk, dw, dY, d_status=None, opts=None, stream=None) -> int:
    return lib.kgev_eigh_device(ctx.handle, _ptr(dA), n, lda, nk, _ptr(dw), _ptr(dY), _ptr(d_status),
                                None if opts is None else ctypes.byref(opts), _stream(stream))


def zgemm_device(ctx, transa, transb, m, n, k, alpha, dA, lda, sA, dB, ldb, sB, beta, dC, ldc, sC, batch,
                 lower=False, stream=None) -> int:
    al, be = complex(alpha), complex(beta)
    return lib.kgev_zgemm_device(ctx.handle, transa.encode(), transb.encode(), m, n, k, Z(al.real, al.imag),
                                 _ptr(dA), lda, sA, _ptr(dB), ldb, sB, Z(be.real, be.imag), _ptr(dC), ldc, sC,
                                 batch, 1 if lower else 0, _stream(stream))


def fermi_device(ctx, dw, n, nk, d_wk, nelec, kT, g, d_occ, d_result, d_status, ldw=None, ldo=None,
                 stream=None) -> int:
    """kgev_fermi_device: Band_DFT_Col Part 5 (mu, band energy, occupations)."""
    return lib.kgev_fermi_device(ctx.handle, _ptr(dw), n if ldw is None else ldw, n, nk, _ptr(d_wk), float(nelec),
                                 float(kT), float(g), _ptr(d_occ), n if ldo is None else ldo, _ptr(d_result),
                                 _ptr(d_status), _stream(stream))


def density_workspace_bytes(n, nk, nocc) -> int:
    return lib.kgev_density_workspace_bytes(n, nk, nocc)


def density_device(ctx, dC, n, nk, nocc, dw, d_occ, d_wk, g, d_rho, d_edm=None, ldc=None, ldw=None, ldo=None,
                   ldr=None, dwork=None, work_bytes=0, stream=None) -> int:
    """kgev_density_device: Band_DFT_Col Part 6 (charge and energy density
    matrices, lower triangles)."""
    return lib.kgev_density_device(ctx.handle, _ptr(dC), n if ldc is None else ldc, n, nk, nocc, _ptr(dw),
                                   n if ldw is None else ldw, _ptr(d_occ), n if ldo is None else ldo, _ptr(d_wk),
                                   float(g), _ptr(d_rho), _ptr(d_edm), n if ldr is None else ldr, _ptr(dwork),
                                   int(work_bytes), _stream(stream))


def bloch_device(ctx, off, blocks, d_data, R, kf, d_out, stream=None) -> int:
    """kgev_bloch_device: Band_DFT_Col Part 1.  ``blocks`` is a list of
    (I, J, r, doff) sorted by (I, J) with the block data at d_data + doff;
    off, R (nR x 3) and kf (nk x 3) are host arrays."""
    import numpy as np
    off = np.ascontiguousarray(off, dtype=np.int32)
    bi = np.ascontiguousarray([b[0] for b in blocks], dtype=np.int32)
    bj = np.ascontiguousarray([b[1] for b in blocks], dtype=np.int32)
    rid = np.ascontiguousarray([b[2] for b in blocks], dtype=np.int32)
    doff = np.ascontiguousarray([b[3] for b in blocks], dtype=np.int64)
    R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1, 3)
    kf = np.ascontiguousarray(kf, dtype=np.float64).reshape(-1, 3)
    hp = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else None
    return lib.kgev_bloch_device(ctx.handle, len(off) - 1, hp(off), len(blocks), hp(bi), hp(bj), hp(rid), hp(doff),
                                 _ptr(d_data), d_data.numel(), len(R), hp(R), len(kf), hp(kf), _ptr(d_out),
                                 _stream(stream))


def profile_begin(ctx, phase, stride: int = 1) -> None:
    _check("kgev_profile_begin", lib.kgev_profile_begin(ctx.handle, int(phase), int(stride)))


def profile_end(ctx):
    """Returns dict(launches, phase_launches, ms, bytes, flops): the timed
    launches, all launches of the phase, and the duration and algorithmic
    work of the timed ones."""
    n, na = ctypes.c_int64(), ctypes.c_int64()
    ms, by, fl = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check("kgev_profile_end", lib.kgev_profile_end(ctx.handle, ctypes.byref(n), ctypes.byref(na),
                                                    ctypes.byref(ms), ctypes.byref(by), ctypes.byref(fl)))
    return dict(launches=n.value, phase_launches=na.value, ms=ms.value, bytes=by.value, flops=fl.value)


class Server:
    """kgev_server: continuous-batching request loop on one device."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, max_slots: int = 4):
        h = ctypes.c_void_p()
        _check("kgev_server_create", lib.kgev_server_create(ctypes.byref(h), int(device), int(hbm_budget),
                                                            int(max_slots)))
        self.handle = h

    def submit(self, dH, dS, n, nk, dw, dC=None, ld=None, ldc=None, precision=PREC_FP64) -> int:
        rq = Request(n, nk, ld or n, _ptr(dH), _ptr(dS), _ptr(dw), _ptr(dC), ldc or n, precision, 0)
        t = ctypes.c_uint64()
        _check("kgev_server_submit", lib.kgev_server_submit(self.handle, ctypes.byref(rq), ctypes.byref(t)))
        return t.value

    def set_bypass(self, max_bypass: int):
        _check("kgev_server_set_bypass", lib.kgev_server_set_bypass(self.handle, int(max_bypass)))

    def poll(self, ticket) -> bool:
        d = ctypes.c_int32()
        _check("kgev_server_poll", lib.kgev_server_poll(self.handle, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket) -> Result:
        r = Result()
        _check("kgev_server_wait", lib.kgev_server_wait(self.handle, ticket, ctypes.byref(r)))
        return r

    def close(self):
        if self.handle:
            lib.kgev_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def autotune(ctx, n, precision=PREC_FP64) -> int:
    best = ctypes.c_int32()
    _check("kgev_autotune", lib.kgev_autotune(ctx.handle, int(n), int(precision), ctypes.byref(best)))
    return best.value


def tuned_params(ctx, n, precision=PREC_FP64):
    """(panel_nb, hemv_slots, gemm_slots, tuned) that solves of order n use
    through ctx when the options leave them 0."""
    nb, hs, gs, tuned = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check("kgev_tuned_params", lib.kgev_tuned_params(ctx.handle, int(n), int(precision), ctypes.byref(nb),
                                                       ctypes.byref(hs), ctypes.byref(gs), ctypes.byref(tuned)))
    return nb.value, hs.value, gs.value, bool(tuned.value)
