"""Parity of the exact top level and the coarse-route contractions at the
shapes the benchmark and the largest configuration use: many coarse sites
per time row (each of the site ranges that split a row holds several
sites), N_v^2 > 64 (the lanes of a wavefront loop over the N_v x N_v
entries of (gamma5 gamma_k)_1), r = 2 N_lm = 32 (two column tiles, two row
chunks) and r = 128 (the largest top level), against eq:G_LL:exact and the
fine-route contraction of the prolonged vectors in the oracle."""
import numpy as np
import pytest

from oracle import coarse, estimators as est
from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, relerr
from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rows256():
    # 128 coarse sites per time row, N_v = 24 (n_c = 48), N_lm = 16 (r = 32)
    return Pair((4, 8, 8, 16), (2, 2, 2, 2), 24, kappa=0.124, Nlm=16)


def test_top_level_many_sites_per_row(rows256):
    P = rows256
    assert P.bl.V1 // P.bl.L1[0] == 128 and P.ctx.r == 32
    G1 = coarse.coarse_gammas(P.B)
    ref = est.exact_top(P.top.Q2, P.top.gammas(G1, P.bl), P.L)
    got = P.ctx.contract_top()
    err = relerr(got, ref)
    print("exact top, r = 32, 128 coarse sites per row: %.2e" % err)
    assert err < 1e-10


def test_coarse_route_nv24(rows256):
    """Coarse contractions with N_v = 24 (per-slice chunks of the level
    assembly and the single-source calls) against the oracle's fine route."""
    P = rows256
    nc = 2 * P.Nv
    ci = synth.gaussian_coarse(12, P.bl.V1, nc, 81)
    cj = synth.gaussian_coarse(12, P.bl.V1, nc, 82)
    fi, fj = P.B.prolong(ci), P.B.prolong(cj)
    ref = est.point_correlator(fi, fj, 3)
    assert relerr(P.ctx.contract_point_coarse(to_dev(ci), to_dev(cj), 3), ref) < 1e-12
    assert relerr(P.ctx.contract_pair(0, [3], to_dev(ci), to_dev(cj), coarse=True), ref) < 1e-12
    ref = est.stochastic_pair(fi[:4], fj[:4], 2, P.L)
    assert relerr(P.ctx.contract_stoch_coarse(to_dev(ci[:4]), to_dev(cj[:4]), 2), ref) < 1e-12


def test_top_level_r128():
    """N_v = 32, N_lm = 64: the largest top level (eight column tiles and
    eight row chunks of 16)."""
    P = Pair((4, 4, 4, 8), (2, 2, 2, 2), 32, kappa=0.124, Nlm=64)
    assert P.ctx.r == 128
    G1 = coarse.coarse_gammas(P.B)
    ref = est.exact_top(P.top.Q2, P.top.gammas(G1, P.bl), P.L)
    got = P.ctx.contract_top()
    err = relerr(got, ref)
    print("exact top, r = 128: %.2e" % err)
    assert err < 1e-10
