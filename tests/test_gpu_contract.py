"""GPU parity of sources and contractions (point, stochastic, coarse route,
exact top level) against the oracle, and the whole two-/three-level point
source pipeline on the 4^4 workload against the oracle's dense propagators."""
import numpy as np
import pytest

from oracle import dirac, coarse, estimators as est
from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, from_dev, relerr
from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pair():
    # the 4^4 workload: 2^4 blocks, 8 test vectors, 4 top modes
    return Pair((4, 4, 4, 4), (2, 2, 2, 2), 8, kappa=0.120, Nlm=4)


@pytest.fixture(scope="module")
def pair2():
    return Pair((8, 4, 2, 6), (4, 2, 2, 3), 3, kappa=0.124, Nlm=2)


@pytest.mark.parametrize("which", ["pair", "pair2"])
def test_point_contraction_parity(which, request):
    P = request.getfixturevalue(which)
    Si = synth.gaussian_fields(12, P.L, 11)
    Sj = synth.gaussian_fields(12, P.L, 12)
    for y0 in (0, P.L[0] - 1):
        ref = est.point_correlator(P.lat(Si), P.lat(Sj), y0)
        got = P.ctx.contract_point(P.fine_dev(Si), P.fine_dev(Sj), y0)
        assert relerr(got, ref) < 1e-12


@pytest.mark.parametrize("which", ["pair", "pair2"])
def test_stochastic_contraction_parity(which, request):
    P = request.getfixturevalue(which)
    Si = synth.gaussian_fields(4, P.L, 13)
    Sj = synth.gaussian_fields(4, P.L, 14)
    tn = 1
    ref = est.stochastic_pair(P.lat(Si), P.lat(Sj), tn, P.L)
    got = P.ctx.contract_stoch(P.fine_dev(Si), P.fine_dev(Sj), tn)
    assert relerr(got, ref) < 1e-12


@pytest.mark.parametrize("which", ["pair", "pair2"])
def test_coarse_route_equals_fine_route(which, request):
    """The coarse contraction through (gamma5 gamma_k)_1 equals the oracle's
    fine contraction of the prolonged vectors."""
    P = request.getfixturevalue(which)
    nc = 2 * P.Nv
    ci = synth.gaussian_coarse(12, P.bl.V1, nc, 15)
    cj = synth.gaussian_coarse(12, P.bl.V1, nc, 16)
    ref = est.point_correlator(P.B.prolong(ci), P.B.prolong(cj), 2)
    got = P.ctx.contract_point_coarse(to_dev(ci), to_dev(cj), 2)
    assert relerr(got, ref) < 1e-12
    ref = est.stochastic_pair(P.B.prolong(ci[:4]), P.B.prolong(cj[:4]), 1, P.L)
    got = P.ctx.contract_stoch_coarse(to_dev(ci[:4]), to_dev(cj[:4]), 1)
    assert relerr(got, ref) < 1e-12


@pytest.mark.parametrize("which", ["pair", "pair2"])
def test_exact_top_parity(which, request):
    P = request.getfixturevalue(which)
    G1 = coarse.coarse_gammas(P.B)
    ref = est.exact_top(P.top.Q2, P.top.gammas(G1, P.bl), P.L)
    got = P.ctx.contract_top()
    assert relerr(got, ref) < 1e-10


def test_sources_parity(pair):
    import torch
    L = pair.L
    out = pair.ctx.fine(12)
    pair.ctx.point_sources((1, 2, 3, 0), out)
    ref = pair.canon(est.point_sources(L, (1, 2, 3, 0)))
    assert np.array_equal(pair.fine_host(out), ref)
    xi = synth.z4_noise(2, L, 3)
    t = synth.time_slices(2, L[0], 4)
    out = pair.ctx.fine(8)
    pair.ctx.noise_sources(to_dev(xi), t, out)
    got = pair.fine_host(out)
    for n in range(2):
        ref = pair.canon(est.spin_diluted_sources(L, xi[n], t[n]))
        assert np.array_equal(got[4 * n:4 * n + 4], ref)


def test_point_source_pipeline(pair):
    """Three-level decomposition of the point-source correlator on the 4^4
    workload: GPU solve + coarse pieces + contractions against the oracle's
    dense propagators, level by level, and the sum against the full C."""
    import torch
    from paper_2412_06347_amd import mglma
    L, ctx = pair.L, pair.ctx
    V = int(np.prod(L))
    # oracle: dense propagators and pieces
    S = np.linalg.inv(pair.D.dense())
    T = pair.B.basis_canonical().reshape(pair.bl.V1 * 2 * pair.Nv, -1).T
    A1 = coarse.coarse_dense(pair.D1, pair.nbr)
    Sge1 = T @ np.linalg.inv(A1) @ T.conj().T
    W = pair.top.W
    S2 = T @ W @ np.linalg.inv(pair.top.D2) @ W.conj().T @ T.conj().T
    y = (0, 0, 0, 0)
    cols = lambda M: np.stack([M[:, a].reshape(*L, 4, 3) for a in range(12)])
    full, ge1, top = cols(S), cols(Sge1), cols(S2)
    ref_all = est.point_correlator(full, full, 0)
    ref_ge1 = est.point_correlator(ge1, ge1, 0)
    ref_top = est.point_correlator(top, top, 0)
    # GPU
    src = ctx.fine(12)
    ctx.point_sources(y, src)
    x = ctx.fine(12)
    p = mglma.default_params(inner=mglma.F32, coarse=mglma.BF16, tol=1e-11)
    ctx.solve(src, x, p)
    cg = ctx.coarse(12)
    ct = ctx.coarse(12)
    ctx.coarse_pieces(src, cg, ct, p)
    got_all = ctx.contract_point(x, x, 0)
    got_ge1 = ctx.contract_point_coarse(cg, cg, 0)
    got_top = ctx.contract_point_coarse(ct, ct, 0)
    assert relerr(got_all, ref_all) < 1e-9
    assert relerr(got_ge1, ref_ge1) < 1e-9
    assert relerr(got_top, ref_top) < 1e-9
    # level sums by bilinearity: G_L0 = C(S,S) - C(S>=1,S>=1), G_L1 = C(S>=1,S>=1) - C(S2,S2)
    assert relerr(got_all - got_ge1, ref_all - ref_ge1) < 1e-8
