"""The allocation-free level assembly (mglma_contract_levels_noalloc, fixed
device workspace) against mglma_contract_levels on the same inputs: two
calls in a row, the second with a smaller input, and a call whose sources
need two passes through the fixed workspace."""
import numpy as np
import pytest

from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev
from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu

STOCH, POINT = 1, 0


def close(a, b, tol):
    return np.abs(a - b).max() <= tol * np.abs(b).max()


def test_noalloc_matches_levels_twice():
    P = Pair((4, 4, 4, 4), (2, 2, 2, 2), 8, kappa=0.120)
    ctx, L, nc = P.ctx, P.L, 2 * P.Nv
    # first call: 5 stochastic sources, a fine and two coarse pieces
    tn = [0, 3, 1, 2, 3]
    f = P.fine_dev(synth.gaussian_fields(20, L, 201))
    c1 = to_dev(synth.gaussian_coarse(20, P.bl.V1, nc, 202))
    c2 = to_dev(synth.gaussian_coarse(20, P.bl.V1, nc, 203))
    ref = ctx.contract_levels(STOCH, tn, fine=f, coarse=[c1, c2])
    got = ctx.contract_levels_noalloc(STOCH, tn, fine=f, coarse=[c1, c2])
    assert got.shape == (3, L[0]) and close(got, ref, 1e-14)
    # second call, smaller: 2 point sources, one coarse piece
    c3 = to_dev(synth.gaussian_coarse(24, P.bl.V1, nc, 204))
    ref = ctx.contract_levels(POINT, [1, 2], coarse=[c3])
    got = ctx.contract_levels_noalloc(POINT, [1, 2], coarse=[c3])
    assert got.shape == (1, L[0]) and close(got, ref, 1e-14)


def test_noalloc_two_passes():
    """L0 = 64 with three pieces: the fixed workspace holds 85 sources per
    pass, so 100 sources take two passes."""
    P = Pair((64, 2, 2, 2), (2, 2, 2, 2), 4, kappa=0.120)
    ctx, L, nc = P.ctx, P.L, 2 * P.Nv
    nsrc = 100
    tn = synth.time_slices(nsrc, L[0], 205)
    f = P.fine_dev(synth.gaussian_fields(4 * nsrc, L, 206))
    c1 = to_dev(synth.gaussian_coarse(4 * nsrc, P.bl.V1, nc, 207))
    c2 = to_dev(synth.gaussian_coarse(4 * nsrc, P.bl.V1, nc, 208))
    ref = ctx.contract_levels(STOCH, tn, fine=f, coarse=[c1, c2])
    got = ctx.contract_levels_noalloc(STOCH, tn, fine=f, coarse=[c1, c2])
    assert close(got, ref, 1e-13)
    # a smaller call afterwards reads nothing the previous call left behind
    ref = ctx.contract_levels(STOCH, tn[:3], coarse=[c1[:12], c2[:12]])
    got = ctx.contract_levels_noalloc(STOCH, tn[:3], coarse=[c1[:12], c2[:12]])
    assert close(got, ref, 1e-14)
