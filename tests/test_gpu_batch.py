"""Systems of uneven order in one call (kgev_solve_batch_device): every
problem's eigenvalues and vectors are bitwise those of its own
kgev_solve_k_device call with the same options, and match the oracle; the
captured-graph form replays to the same results (with the program's own work
and synchronisations between replays); bad descriptors and a short workspace
are rejected."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, K, check, dev, host, residuals

pytestmark = pytest.mark.gpu

from paper_1402_4247_amd import inputs as G  # noqa: E402


def systems():
    out = []
    for n, nk, seed in [(70, 2, 31), (130, 1, 32), (33, 3, 33), (1, 2, 34)]:
        Hs, Ss = G.config1_batch(n, nk, seed)
        out.append((n, nk, Hs, Ss))
    return out


def buffers(n, nk):
    return (torch.zeros((nk, n), dtype=torch.float64, device=DEV),
            torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV),
            torch.full((nk,), -9, dtype=torch.int32, device=DEV))


def test_batch_equals_single_calls_and_oracle():
    kg = K()
    sy = systems()
    dev_in = [(dev(Hs), dev(Ss)) for _, _, Hs, Ss in sy]
    with kg.Context(0) as ctx:
        outs, probs = [], []
        for (n, nk, _, _), (dH, dS) in zip(sy, dev_in):
            w, C, st = buffers(n, nk)
            outs.append((w, C, st))
            probs.append(kg.problem(dH, dS, n, n, nk, w, C, n, st))
        check(kg.solve_batch_device(ctx, probs), "batch")
        torch.cuda.synchronize()
        for (n, nk, Hs, Ss), (dH, dS), (w, C, st) in zip(sy, dev_in, outs):
            w1, C1, st1 = buffers(n, nk)
            check(kg.solve_k_device(ctx, dH, dS, n, n, nk, w1, C1, n, d_status=st1), "single")
            torch.cuda.synchronize()
            assert torch.equal(w, w1) and torch.equal(C, C1) and torch.equal(st, st1)
            assert bool((st == 0).all())
            wh, Ch = w.cpu().numpy(), host(C)
            for q in range(nk):
                s0, w0, _ = O.solve_k(Hs[q], Ss[q])
                assert s0 == 0
                assert np.abs(wh[q] - w0).max() <= 1e-10 * max(np.abs(w0).max(), 1e-300)
                r_res, r_orth = residuals(Hs[q], Ss[q], wh[q], Ch[q])
                assert r_res <= 1e-12 and r_orth <= 1e-12


def test_batch_graph_replays():
    kg = K()
    sy = systems()[:3]
    dev_in = [(dev(Hs), dev(Ss)) for _, _, Hs, Ss in sy]
    stream = torch.cuda.Stream()
    with kg.Context(0) as ctx:
        ref, outs, probs = [], [], []
        for (n, nk, _, _), (dH, dS) in zip(sy, dev_in):
            w, C, st = buffers(n, nk)
            check(kg.solve_k_device(ctx, dH, dS, n, n, nk, w, C, n, d_status=st), "single")
            ref.append((w, C))
            w2, C2, st2 = buffers(n, nk)
            outs.append((w2, C2, st2))
            probs.append(kg.problem(dH, dS, n, n, nk, w2, C2, n, st2))
        torch.cuda.synchronize()
        opts = kg.make_opts(use_graph=True)
        for rep in range(3):
            junk = torch.randn(4096, device=DEV).sum()
            for w2, C2, st2 in outs:
                w2.zero_()
                C2.zero_()
                st2.fill_(-9)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                check(kg.solve_batch_device(ctx, probs, opts=opts, stream=stream.cuda_stream), "graph batch")
            stream.synchronize()
            for (w, C), (w2, C2, st2) in zip(ref, outs):
                assert torch.equal(w, w2) and torch.equal(C, C2), f"replay {rep}"
                assert bool((st2 == 0).all())
            del junk


def test_batch_argument_errors():
    kg = K()
    n, nk = 20, 2
    Hs, Ss = G.config1_batch(n, nk, 5)
    dH, dS = dev(Hs), dev(Ss)
    w, C, st = buffers(n, nk)
    good = kg.problem(dH, dS, n, n, nk, w, C, n, st)
    with kg.Context(0) as ctx:
        assert kg.solve_batch_device(ctx, []) == -3
        bad = kg.problem(dH, dS, n, n - 1, nk, w, C, n, st)          # ld < n
        assert kg.solve_batch_device(ctx, [good, bad]) == -1001
        novec = kg.problem(dH, dS, n, n, nk, w, None, 0, st)
        assert kg.solve_batch_device(ctx, [novec]) == -1000
        assert kg.solve_batch_device(ctx, [novec], opts=kg.make_opts(want_vectors=False)) == 0
        need = kg.batch_workspace_bytes([good])
        ws = torch.empty(need // 8 + 1, dtype=torch.float64, device=DEV)
        assert kg.solve_batch_device(ctx, [good], dwork=ws, work_bytes=need - 1) == -4
        assert kg.solve_batch_device(ctx, [good], dwork=ws, work_bytes=need) == 0
        torch.cuda.synchronize()
        assert bool((st == 0).all())
