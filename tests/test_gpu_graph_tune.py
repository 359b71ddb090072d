"""HIP-graph mode (the whole batched solve captured once and replayed) and the
autotuner (panel width and Hermitian-product tile grouping).  Every graph replay is checked against the eager
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
        assert kg.tuned_params(ctx, n) == (32, 768, 256, False)
        best = kg.autotune(ctx, n)
        assert best in (16, 24, 32, 48, 64)
        nb_t, slots_t, gemm_t, tuned = kg.tuned_params(ctx, n)
        assert tuned and nb_t == best and slots_t in (1, 256, 768, 2048, 1 << 30)
        assert gemm_t in (1, 64, 256, 1024, 1 << 30)
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


@pytest.mark.parametrize("slots", [1, 1 << 30])
def test_hermitian_product_forms_match_oracle(slots):
    """Both tile groupings of the Hermitian product (four 64 x 64 tiles per
    workgroup, hemv_slots = 1; one tile per workgroup, hemv_slots = 2^30) at
    orders with ragged last tiles, against the oracle."""
    import oracle as O
    from gpu_helpers import host
    kg = K()
    for n, nk in ((200, 2), (333, 1)):
        Hs, Ss = G.config2(n, nk, 2002)
        w = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
        C = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
        st = torch.zeros(nk, dtype=torch.int32, device=DEV)
        with kg.Context(0) as ctx:
            run(ctx, dev(Hs), dev(Ss), n, nk, w, C, st, kg.make_opts(hemv_slots=slots))
            torch.cuda.synchronize()
        assert bool((st == 0).all())
        wg, Cg = w.cpu().numpy(), host(C)
        for q in range(nk):
            s0, w0, _ = O.solve_k(Hs[q], Ss[q])
            assert s0 == 0
            assert np.abs(wg[q] - w0).max() <= 1e-10 * np.abs(w0).max()
            r_res = np.linalg.norm(Hs[q] @ Cg[q] - Ss[q] @ Cg[q] * wg[q]) / np.linalg.norm(Hs[q])
            r_orth = np.abs(Cg[q].conj().T @ Ss[q] @ Cg[q] - np.eye(n)).max()
            assert r_res <= 1e-12 and r_orth <= 1e-12


def test_product_tile_sizes_give_the_same_bits():
    """The complex products in 32 x 32 tiles (gemm_slots = 2^30) and in
    64 x 64 tiles (gemm_slots = 1) accumulate every entry in the same order,
    so a whole solve gives the same bits either way (n = 190: ragged tiles of
    both sizes; 2 k-points)."""
    kg = K()
    n, nk = 190, 2
    Hs, Ss = G.config2(n, nk, 2002)
    outs = []
    with kg.Context(0) as ctx:
        for gs in (1, 1 << 30):
            w = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
            C = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
            st = torch.zeros(nk, dtype=torch.int32, device=DEV)
            run(ctx, dev(Hs), dev(Ss), n, nk, w, C, st, kg.make_opts(gemm_slots=gs))
            torch.cuda.synchronize()
            assert bool((st == 0).all())
            outs.append((w.cpu(), C.cpu()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
