"""The C-ABI library loads on any host, exports every entry point that
include/kgev.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1402_4247_amd import kgev as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "kgev.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kgev_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(K.lib, name), name
    assert set(names) == set(K.EXPORTS)
    assert "kgev_server_submit" in names


def test_library_is_the_in_tree_build():
    assert os.path.dirname(K.LIB_PATH) == os.path.join(ROOT, "paper_1402_4247_amd")


def test_status_strings_and_defaults():
    assert K.status_str(0) == "ok"
    assert "positive definite" in K.status_str(1)
    assert "converge" in K.status_str(2)
    assert "non-finite" in K.status_str(3)
    o = K.make_opts()
    assert o.precision == 0 and o.want_vectors == 1 and o.hemv_slots == 0 and o.gemm_slots == 0
    assert all(r == 0 for r in o.reserved)


def test_workspace_bytes_scales_with_problem():
    assert K.workspace_bytes(0, 1) == 0 and K.workspace_bytes(8, 0) == 0
    w1 = K.workspace_bytes(1000, 1)
    w2 = K.workspace_bytes(2000, 1)
    w16 = K.workspace_bytes(2000, 16)
    assert w1 > 0 and 3.5 < w2 / w1 < 4.5 and 15.5 < w16 / w2 < 16.5
    # resident state ~ 4 complex + 3 real n x n matrices per k-point
    assert w2 < 100 * 2000 * 2000


@pytest.mark.parametrize("args,code", [
    # (ctx, H, S, n, ld, nk, w, C, ldc) -> first failing argument
    ((None, 1, 1, 4, 4, 1, 1, 1, 4), -1),
])
def test_null_context_rejected(args, code):
    ctx, H, S, n, ld, nk, w, C, ldc = args
    st = K.lib.kgev_solve_k_device(None, ctypes.c_void_p(H), ctypes.c_void_p(S), n, ld, nk,
                                   ctypes.c_void_p(w), ctypes.c_void_p(C), ldc, None, 0, None, None, None)
    assert st == code


def test_host_api_rejects_null_context():
    bad = ctypes.c_int64(7)
    st = K.lib.kgev_solve_k(None, None, None, 4, 1, None, None, None, ctypes.byref(bad))
    assert st == -1 and bad.value == -1


def test_batch_workspace_covers_the_embedded_class_and_null_ctx_rejected():
    # orders up to 256 form one class of the largest order (here 130) holding
    # all 6 k-points: its solve workspace plus the embedded H, S, C (16 B per
    # entry each), eigenvalues, statuses and column map
    ps = [K.Problem(70, 70, 2), K.Problem(130, 130, 1), K.Problem(33, 40, 3)]
    arr = (K.Problem * 3)(*ps)
    got = K.lib.kgev_batch_workspace_bytes(arr, 3, None)
    N, Kc = 130, 6
    assert got >= K.lib.kgev_workspace_bytes(N, Kc, None) + 3 * 16 * N * N * Kc
    assert got <= K.lib.kgev_workspace_bytes(N, Kc, None) + 3 * 16 * N * N * Kc + 16 * N * Kc + 7 * 256
    # a class of one problem of its own order is solved in place
    one = (K.Problem * 1)(K.Problem(130, 130, 2))
    assert K.lib.kgev_batch_workspace_bytes(one, 1, None) == K.lib.kgev_workspace_bytes(130, 2, None)
    assert K.lib.kgev_batch_workspace_bytes(arr, 0, None) == 0
    assert K.lib.kgev_solve_batch_device(None, arr, 3, None, 0, None, None) == -1


def test_noalloc_entry_rejects_null_context():
    st = K.lib.kgev_solve_k_device_noalloc(None, ctypes.c_void_p(1), ctypes.c_void_p(1), 4, 4, 1,
                                           ctypes.c_void_p(1), ctypes.c_void_p(1), 4, None, None, None)
    assert st == -1


def test_tuned_params_rejects_null_context_and_bad_precision():
    nb, hs, gs, tuned = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert K.lib.kgev_tuned_params(None, 100, 0, ctypes.byref(nb), ctypes.byref(hs), ctypes.byref(gs),
                                   ctypes.byref(tuned)) == -1


def test_driver_is_built_and_rejects_unknown_options():
    import subprocess
    drv = os.path.join(ROOT, "paper_1402_4247_amd", "kgev_driver")
    assert os.path.exists(drv)
    r = subprocess.run([drv, "--bogus", "1"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage" in r.stderr
