"""Concurrent k-point groups (opts.streams): the batch split over several
streams gives bitwise the same eigenvalues, vectors and statuses as one
stream (each k-point's arithmetic does not depend on the grouping), with and
without graph capture, for group counts that do and do not divide nk."""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV, K, check, dev
from paper_1402_4247_amd import inputs as G

pytestmark = pytest.mark.gpu


def solve(ctx, dH, dS, n, nk, opts, stream=None):
    kg = K()
    w = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    C = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    st = torch.full((nk,), -9, dtype=torch.int32, device=DEV)
    check(kg.solve_k_device(ctx, dH, dS, n, n, nk, w, C, n, d_status=st, opts=opts, stream=stream), "solve")
    return w, C, st


@pytest.mark.parametrize("streams", [2, 3, 5])
def test_groups_bitwise_equal_to_one_stream(streams):
    kg = K()
    n, nk = 130, 5
    Hs, Ss = G.config2(n, nk, 2002)
    dH, dS = dev(Hs), dev(Ss)
    with kg.Context(0) as ctx:
        w1, C1, s1 = solve(ctx, dH, dS, n, nk, kg.make_opts(streams=1))
        torch.cuda.synchronize()
        w2, C2, s2 = solve(ctx, dH, dS, n, nk, kg.make_opts(streams=streams))
        torch.cuda.synchronize()
    assert torch.equal(w1, w2) and torch.equal(C1, C2) and torch.equal(s1, s2)
    assert bool((s1 == 0).all())


def test_groups_mixed_precision_and_status():
    # a bad k-point in the second group reports its status at its own index
    kg = K()
    n, nk = 70, 4
    Hs, Ss = G.config1_batch(n, nk, 5)
    Ss = Ss.copy()
    Ss[3] = -Ss[3]                       # not positive definite
    dH, dS = dev(Hs), dev(Ss)
    with kg.Context(0) as ctx:
        for prec in (kg.PREC_FP64, kg.PREC_FP32_REFINE):
            w1, C1, s1 = solve(ctx, dH, dS, n, nk, kg.make_opts(precision=prec, streams=1))
            w2, C2, s2 = solve(ctx, dH, dS, n, nk, kg.make_opts(precision=prec, streams=2))
            torch.cuda.synchronize()
            assert s1.cpu().tolist() == [0, 0, 0, 1] and torch.equal(s1, s2)
            assert torch.equal(w1[:3], w2[:3]) and torch.equal(C1[:3], C2[:3])


def test_groups_under_graph_capture():
    kg = K()
    n, nk = 96, 4
    Hs, Ss = G.config2(n, nk, 2002)
    dH, dS = dev(Hs), dev(Ss)
    stream = torch.cuda.Stream()
    with kg.Context(0) as ctx:
        w1, C1, _ = solve(ctx, dH, dS, n, nk, kg.make_opts(streams=1))
        torch.cuda.synchronize()
        w = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
        C = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
        st = torch.zeros(nk, dtype=torch.int32, device=DEV)
        opts = kg.make_opts(use_graph=True, streams=2)
        for rep in range(3):
            junk = torch.randn(1000, device=DEV).sum()
            torch.cuda.synchronize()
            w.zero_()
            C.zero_()
            st.fill_(-9)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                check(kg.solve_k_device(ctx, dH, dS, n, n, nk, w, C, n, d_status=st, opts=opts,
                                        stream=stream.cuda_stream), "graph solve")
            stream.synchronize()
            assert torch.equal(w, w1) and torch.equal(C, C1), f"replay {rep}"
            assert bool((st == 0).all())
            del junk


def test_invalid_stream_count():
    kg = K()
    n, nk = 16, 2
    Hs, Ss = G.config2(n, nk, 2002)
    dH, dS = dev(Hs), dev(Ss)
    w = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    with kg.Context(0) as ctx:
        for bad in (-1, 9):
            o = kg.make_opts(want_vectors=False, streams=bad)
            assert kg.solve_k_device(ctx, dH, dS, n, n, nk, w, None, n, opts=o) == -10
