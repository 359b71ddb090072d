"""kgev_solve_k_device_noalloc (the solve with the library's static per-GPU
workspace, for callers that cannot allocate) against kgev_solve_k_device on
the same inputs and options: bitwise the same eigenvalues, eigenvectors and
statuses, on two calls in a row, the second one smaller (the static array
keeps the first call's contents), and the oracle on one k-point.  Also: a
size whose workspace exceeds the array is rejected before anything runs."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import DEV, K, check, dev, host, residuals
from paper_1402_4247_amd import inputs as G

pytestmark = pytest.mark.gpu


def both(ctx, Hs, Ss, opts):
    kg = K()
    nk, n = Hs.shape[0], Hs.shape[1]
    dH, dS = dev(Hs), dev(Ss)
    out = []
    for fn in (kg.solve_k_device, kg.solve_k_device_noalloc):
        dw = torch.full((nk, n), np.nan, dtype=torch.float64, device=DEV)
        dC = torch.full((nk, n, n), np.nan, dtype=torch.complex128, device=DEV)
        st = torch.full((nk,), -7, dtype=torch.int32, device=DEV)
        check(fn(ctx, dH, dS, n, n, nk, dw, dC, n, d_status=st, opts=opts), fn.__name__)
        torch.cuda.synchronize()
        out.append((dw, dC, st))
    return out


@pytest.mark.parametrize("form", [{}, {"precision": 1}])
def test_noalloc_equals_allocating_entry_two_calls(form):
    kg = K()
    with kg.Context(0) as ctx:
        opts = kg.make_opts(**form)
        # first call: LCAO pencils n = 300, 3 k-points
        Hs, Ss = G.config2(300, 3, 2002)
        (w1, C1, s1), (w2, C2, s2) = both(ctx, Hs, Ss, opts)
        assert torch.equal(s1, s2) and bool((s1 == 0).all())
        assert torch.equal(w1, w2) and torch.equal(C1, C2)
        st0, w0, _ = O.solve_k(Hs[1], Ss[1])
        assert st0 == 0
        assert np.abs(w2[1].cpu().numpy() - w0).max() <= 1e-10 * np.abs(w0).max()
        rr, ro = residuals(Hs[1], Ss[1], w2[1].cpu().numpy(), host(C2)[1])
        assert rr <= 1e-12 and ro <= 1e-12
        # second call, smaller: dense pencils n = 97, 2 k-points, one of
        # them with an indefinite overlap (status, other k unaffected)
        Hs, Ss = G.config1_batch(97, 2, 4242)
        Ss[0] = np.eye(97)
        Ss[0][5, 5] = -1.0
        (w1, C1, s1), (w2, C2, s2) = both(ctx, Hs, Ss, opts)
        assert torch.equal(s1, s2) and s2.tolist() == [1, 0]
        assert torch.equal(w1[1], w2[1]) and torch.equal(C1[1], C2[1])
        st0, w0, _ = O.solve_k(Hs[1], Ss[1])
        assert np.abs(w2[1].cpu().numpy() - w0).max() <= 1e-10 * np.abs(w0).max()


def test_noalloc_rejects_oversized_and_graph_options():
    kg = K()
    n = 1200
    assert kg.workspace_bytes(n, 1) > kg.NOALLOC_SCRATCH_BYTES
    dH = torch.zeros((1, n, n), dtype=torch.complex128, device=DEV)
    dw = torch.zeros((1, n), dtype=torch.float64, device=DEV)
    with kg.Context(0) as ctx:
        assert kg.solve_k_device_noalloc(ctx, dH, dH, n, n, 1, dw, dH, n) == -9
        o = kg.make_opts(use_graph=True)
        assert kg.solve_k_device_noalloc(ctx, dH[:, :8, :8], dH[:, :8, :8], 8, 8, 1, dw, dH, 8, opts=o) == \
            kg.EUNSUPPORTED
    torch.cuda.synchronize()
