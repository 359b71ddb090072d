"""Admission policy of the serving loop (the product's ServeCore), exercised
on the host with a stand-in executor: arrival order, HBM budget and slot
limits are never exceeded, queued work starts as soon as resources free up,
requests that can never fit are rejected, a request that fails to start does
not block the others; with bounded bypass, later requests that fit start ahead
of a head that does not, never more often than the bound."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
QUEUED, RUNNING, DONE = 0, 1, 2


@pytest.fixture(scope="module")
def H():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "serve_harness.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-Wall",
                           "-I", os.path.join(ROOT, "paper_1402_4247_amd", "csrc"),
                           os.path.join(HERE, "serve_harness.cpp"), "-o", so])
    lib = ctypes.CDLL(so)
    lib.sh_create.restype = ctypes.c_void_p
    lib.sh_create.argtypes = [ctypes.c_uint64, ctypes.c_int]
    for f in ["sh_destroy"]:
        getattr(lib, f).argtypes = [ctypes.c_void_p]
    lib.sh_submit.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
    lib.sh_set_bypass.argtypes = [ctypes.c_void_p, ctypes.c_int]
    for f in ["sh_step", "sh_max_running", "sh_running"]:
        getattr(lib, f).argtypes = [ctypes.c_void_p]
    for f in ["sh_state", "sh_start_seq", "sh_failed"]:
        getattr(lib, f).argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.sh_peak_bytes.argtypes = [ctypes.c_void_p]
    lib.sh_peak_bytes.restype = ctypes.c_uint64
    lib.sh_in_use.argtypes = [ctypes.c_void_p]
    lib.sh_in_use.restype = ctypes.c_uint64
    return lib


def run_to_completion(lib, h, ids, max_steps=10000):
    for _ in range(max_steps):
        lib.sh_step(h)
        if all(lib.sh_state(h, i) == DONE for i in ids):
            return
    raise AssertionError("did not drain")


def test_fifo_budget_and_slots(H):
    h = H.sh_create(100, 3)
    rng = np.random.default_rng(0)
    ids = [H.sh_submit(h, int(rng.integers(1, 60)), int(rng.integers(1, 8)), 0) for _ in range(40)]
    assert all(i >= 0 for i in ids)
    run_to_completion(H, h, ids)
    seq = [H.sh_start_seq(h, i) for i in ids]
    assert seq == sorted(seq) == list(range(40))          # started in arrival order
    assert H.sh_max_running(h) <= 3
    assert H.sh_peak_bytes(h) <= 100
    assert H.sh_in_use(h) == 0 and H.sh_running(h) == 0
    H.sh_destroy(h)


def test_never_fitting_request_is_rejected(H):
    h = H.sh_create(100, 2)
    assert H.sh_submit(h, 101, 1, 0) == -1
    ok = H.sh_submit(h, 100, 1, 0)
    assert ok >= 0
    run_to_completion(H, h, [ok])
    H.sh_destroy(h)


def test_continuous_admission(H):
    # a long request holds a slot; short ones keep flowing through the other
    h = H.sh_create(100, 2)
    long_id = H.sh_submit(h, 50, 1000, 0)
    short = [H.sh_submit(h, 50, 2, 0) for _ in range(5)]
    H.sh_step(h)
    assert H.sh_state(h, long_id) == RUNNING and H.sh_state(h, short[0]) == RUNNING
    for _ in range(30):
        H.sh_step(h)
    assert all(H.sh_state(h, i) == DONE for i in short)   # done while the long one runs
    assert H.sh_state(h, long_id) == RUNNING
    run_to_completion(H, h, [long_id])
    H.sh_destroy(h)


def test_head_of_line_waits_for_memory(H):
    h = H.sh_create(100, 4)
    a = H.sh_submit(h, 70, 5, 0)
    b = H.sh_submit(h, 70, 1, 0)        # must wait for a (memory), even with free slots
    c = H.sh_submit(h, 10, 1, 0)        # arrival order keeps c behind b
    H.sh_step(h)
    assert H.sh_state(h, a) == RUNNING and H.sh_state(h, b) == QUEUED and H.sh_state(h, c) == QUEUED
    run_to_completion(H, h, [a, b, c])
    assert H.sh_start_seq(h, a) < H.sh_start_seq(h, b) < H.sh_start_seq(h, c)
    H.sh_destroy(h)


def test_failed_start_is_isolated(H):
    h = H.sh_create(100, 2)
    ids = [H.sh_submit(h, 30, 2, 1 if q == 2 else 0) for q in range(6)]
    run_to_completion(H, h, ids)
    assert [H.sh_failed(h, i) for i in ids] == [0, 0, 1, 0, 0, 0]
    assert H.sh_in_use(h) == 0
    H.sh_destroy(h)


def test_bypass_fills_memory_but_bounds_the_head(H):
    # budget 100, 4 slots: A (70) runs long; the head B (50) does not fit
    # beside it, C, D, E (10 each) do.  Strict order keeps them behind B;
    # bypass 2 lets exactly two of them pass B, and B then starts before E.
    for k, passed in [(0, 0), (2, 2), (8, 3)]:
        h = H.sh_create(100, 4)
        H.sh_set_bypass(h, k)
        ids = [H.sh_submit(h, 70, 6, 0), H.sh_submit(h, 50, 2, 0)]
        ids += [H.sh_submit(h, 10, 2, 0) for _ in range(3)]
        run_to_completion(H, h, ids)
        seq = [H.sh_start_seq(h, i) for i in ids]
        a, b, c, d, e = seq
        assert a == 0
        ahead_of_b = sum(1 for x in (c, d, e) if x < b)
        assert ahead_of_b == passed, (k, seq)
        assert c < d < e                      # the small ones keep their order
        assert H.sh_peak_bytes(h) <= 100 and H.sh_max_running(h) <= 4
        H.sh_destroy(h)


def test_bypass_never_starves_and_respects_limits(H):
    rng = np.random.default_rng(3)
    for k in (1, 3):
        h = H.sh_create(120, 3)
        H.sh_set_bypass(h, k)
        sizes = [int(rng.integers(1, 100)) for _ in range(60)]
        ids = [H.sh_submit(h, sz, int(rng.integers(1, 6)), 0) for sz in sizes]
        run_to_completion(H, h, ids)
        seq = [H.sh_start_seq(h, i) for i in ids]
        # request q starts after at most k requests that arrived after it
        for q in range(len(ids)):
            later_first = sum(1 for p in range(q + 1, len(ids)) if seq[p] < seq[q])
            assert later_first <= k * (q + 1), (k, q)
        assert H.sh_peak_bytes(h) <= 120 and H.sh_max_running(h) <= 3
        H.sh_destroy(h)
