"""HIP-graph mode (the whole batched solve captured once and replayed) and the
panel-width autotuner.  Every graph replay is checked against the eager
result, with the program's own eager work and synchronisations between
replays, and with the input buffers rewritten in place between replays."""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV, K, check, dev
from paper_1402_4247_amd import inputs as G

pytestmark = pytest.mark.gpu


def run(ctx, dH, dS, n, nk, w, C, st, opts, stream=None):
    kg = K()
    check(kg.solve_k_device(ctx, dH, dS, n, n, nk, w, C, n, d_status=st, opts=opts, stream=stream), "solve")


def test_graph_replays_match_eager():
    kg = K()
    n, nk = 96, 3
    Hs, Ss = G.config2(n, nk, 2002)
    H2, S2 = G.config1_batch(n, nk, 99)
    dH, dS = dev(Hs), dev(Ss)
    w = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    C = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    st = torch.zeros(nk, dtype=torch.int32, device=DEV)
    stream = torch.cuda.Stream()
    with kg.Context(0) as ctx:
        eager = kg.make_opts()
        graph = kg.make_opts(use_graph=True)
        run(ctx, dH, dS, n, nk, w, C, st, eager)
        torch.cuda.synchronize()
        w_ref, C_ref = w.clone(), C.clone()
        dH2, dS2 = dev(H2), dev(S2)
        run(ctx, dH2, dS2, n, nk, w, C, st, eager)
        torch.cuda.synchronize()
        w_ref2, C_ref2 = w.clone(), C.clone()
        for rep in range(4):
            # eager work of the program between replays
            junk = torch.randn(1000, device=DEV).sum()
            torch.cuda.synchronize()
            w.zero_()
            C.zero_()
            st.fill_(-9)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                run(ctx, dH, dS, n, nk, w, C, st, graph, stream=stream.cuda_stream)
            stream.synchronize()
            assert torch.equal(w, w_ref) and torch.equal(C, C_ref), f"replay {rep}"
            assert bool((st == 0).all())
            del junk
        # same buffers, new contents: the replay reads the current inputs
        dH.copy_(dH2)
        dS.copy_(dS2)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            run(ctx, dH, dS, n, nk, w, C, st, graph, stream=stream.cuda_stream)
        stream.synchronize()
        assert torch.equal(w, w_ref2) and torch.equal(C, C_ref2)


def test_autotune_choice_is_used_and_batch_independent():
    kg = K()
    n = 150
    Hs, Ss = G.config2(n, 2, 2002)
    with kg.Context(0) as ctx:
        best = kg.autotune(ctx, n)
        assert best in (16, 24, 32, 48, 64)
        outs = []
        for nb, k in ((0, 2), (best, 2), (0, 1)):
            w = torch.zeros((k, n), dtype=torch.float64, device=DEV)
            C = torch.zeros((k, n, n), dtype=torch.complex128, device=DEV)
            st = torch.zeros(k, dtype=torch.int32, device=DEV)
            run(ctx, dev(Hs[:k]), dev(Ss[:k]), n, k, w, C, st, kg.make_opts(panel_nb=nb))
            torch.cuda.synchronize()
            outs.append((w.cpu().numpy(), C.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[2][0][0], outs[0][0][0]) and np.array_equal(outs[2][1][0], outs[0][1][0])
