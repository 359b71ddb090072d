"""Kernel timing entry points: with a stride, every stride-th launch of the
phase is timed, all launches are counted, and the algorithmic work tallied is
that of the timed launches (for the Hermitian product, 16 m (m + 1) / 2 bytes
per k-point, m the trailing order of the column).  The Hermitian product is
launched for the columns of the blocked reduction; the last panels, from the
first panel start whose trailing matrix has at most 128 rows, are reduced by
one LDS-resident launch that is not part of the phase."""
import pytest
import torch

from gpu_helpers import DEV, K, check, dev
from paper_1402_4247_amd import inputs as G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("stride", [1, 4, 7])
def test_sampled_hemv_timing(stride):
    kg = K()
    n, nk, nb = 300, 2, 32
    Hs, Ss = G.config1_batch(n, nk, 5)
    dH, dS = dev(Hs), dev(Ss)
    w = torch.zeros((nk, n), dtype=torch.float64, device=DEV)
    C = torch.zeros((nk, n, n), dtype=torch.complex128, device=DEV)
    with kg.Context(0) as ctx:
        kg.profile_begin(ctx, kg.PHASE_HEMV, stride)
        check(kg.solve_k_device(ctx, dH, dS, n, n, nk, w, C, n, opts=kg.make_opts(panel_nb=nb)), "solve")
        prof = kg.profile_end(ctx)
    # two tridiagonalisations (S in Part 2, A in Part 4); blocked columns up to
    # the first panel start p with n - p <= 128
    ptail = next(p for p in range(0, n, nb) if n - p <= 128)
    ms = [n - 1 - i for i in range(ptail)] * 2
    timed = [m for s, m in enumerate(ms) if s % stride == 0]
    assert prof["phase_launches"] == len(ms)
    assert prof["launches"] == len(timed)
    assert prof["bytes"] == sum(16.0 * 0.5 * m * (m + 1) * nk for m in timed)
    assert prof["ms"] > 0


def test_profile_argument_errors():
    kg = K()
    with kg.Context(0) as ctx:
        assert kg.lib.kgev_profile_begin(ctx.handle, kg.PHASE_HEMV, 0) == -3
        assert kg.lib.kgev_profile_begin(ctx.handle, 9, 1) == -2
        assert kg.lib.kgev_profile_end(ctx.handle, None, None, None, None, None) == kg.EUNSUPPORTED
