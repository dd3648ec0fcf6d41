"""GPU solves checked with the oracle: the true FP64 residual ||b - M x||/||b||
is evaluated with the oracle's operator, and small systems are compared with
the oracle's dense solution."""
import numpy as np
import pytest

from oracle import dirac, coarse, solvers
from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, from_dev, relerr
from tests.gpu_setup import Pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pair():
    return Pair((8, 4, 4, 8), (4, 2, 2, 4), 6, kappa=0.124, Nlm=2)


def _true_res(pair, x, b):
    r = pair.canon(pair.D.M(pair.lat(x))) - b
    return np.linalg.norm(r.reshape(len(b), -1), axis=1) / np.linalg.norm(b.reshape(len(b), -1), axis=1)


@pytest.mark.parametrize("mode", ["fp64_gcr", "fp64_mg", "mixed_mg", "mixed_mg_bf16", "mixed_mg_f16smooth",
                                  "fp64_mg_cagcr", "mixed_mg_cagcr", "mixed_mg_f16_cagcr"])
def test_fine_solve(pair, mode):
    from paper_2412_06347_amd import mglma
    kw = dict(tol=1e-10, gcr_m=8, max_inner=400, max_outer=10)
    if mode == "fp64_mg_cagcr":
        kw.update(inner=mglma.F64, coarse=mglma.F64, smoother=mglma.F64, inner_tol=1e-11,
                  smoother_alg=mglma.SMOOTH_CAGCR, nu_post=6)
    elif mode == "mixed_mg_cagcr":
        kw.update(inner=mglma.F32, coarse=mglma.BF16, inner_tol=1e-5, smoother_alg=mglma.SMOOTH_CAGCR, nu_post=4)
    elif mode == "mixed_mg_f16_cagcr":
        kw.update(inner=mglma.F32, coarse=mglma.BF16, smoother=mglma.F16, inner_tol=1e-5,
                  smoother_alg=mglma.SMOOTH_CAGCR, nu_post=8)
    elif mode == "fp64_gcr":
        kw.update(inner=mglma.F64, use_mg=0, inner_tol=1e-11, max_inner=2000, gcr_m=16)
    elif mode == "fp64_mg":
        kw.update(inner=mglma.F64, coarse=mglma.F64, inner_tol=1e-11)
    elif mode == "mixed_mg":
        kw.update(inner=mglma.F32, coarse=mglma.F32, inner_tol=1e-5)
    elif mode == "mixed_mg_bf16":
        kw.update(inner=mglma.F32, coarse=mglma.BF16, inner_tol=1e-5)
    else:
        kw.update(inner=mglma.F32, coarse=mglma.BF16, smoother=mglma.F16, inner_tol=1e-5)
    b = synth.gaussian_fields(3, pair.L, 123)
    bd = pair.fine_dev(b)
    xd = pair.ctx.fine(3)
    rc, stats = pair.ctx.solve(bd, xd, mglma.default_params(**kw), raise_on_error=False)
    x = pair.fine_host(xd)
    res = _true_res(pair, x, b)
    print(mode, "rc", rc, "true rel res", res, "stats", stats)
    assert np.all(res <= 1.05e-10)
    for s in stats:
        assert s["status"] == 0 and s["true_rel_res"] <= 1e-10


def test_solution_matches_oracle_gcr(pair):
    from paper_2412_06347_amd import mglma
    b = synth.gaussian_fields(1, pair.L, 5)
    xo, _, res = solvers.gcr(pair.D.M, pair.lat(b), tol=1e-12)
    bd = pair.fine_dev(b)
    xd = pair.ctx.fine(1)
    pair.ctx.solve(bd, xd, mglma.default_params(inner=mglma.F32, coarse=mglma.BF16, tol=1e-11))
    assert relerr(pair.fine_host(xd), pair.canon(xo)) < 1e-9


@pytest.mark.parametrize("alg", ["mr", "cagcr"])
def test_batch_independence(pair, alg):
    """A right-hand side solved alone and inside a batch gives the same answer
    to the solve tolerance."""
    from paper_2412_06347_amd import mglma
    b = synth.gaussian_fields(4, pair.L, 55)
    p = mglma.default_params(inner=mglma.F32, coarse=mglma.BF16, tol=1e-10)
    if alg == "cagcr":
        p = mglma.default_params(inner=mglma.F32, coarse=mglma.BF16, tol=1e-10, smoother=mglma.F16,
                                 smoother_alg=mglma.SMOOTH_CAGCR, nu_post=8)
    xa = pair.ctx.fine(4)
    pair.ctx.solve(pair.fine_dev(b), xa, p)
    x1 = pair.ctx.fine(1)
    pair.ctx.solve(pair.fine_dev(b[2:3]), x1, p)
    assert relerr(pair.fine_host(xa)[2:3], pair.fine_host(x1)) < 1e-9


def test_coarse_solve_and_pieces(pair):
    import torch
    from paper_2412_06347_amd import mglma
    A = coarse.coarse_dense(pair.D1, pair.nbr)
    v = synth.gaussian_coarse(2, pair.bl.V1, 2 * pair.Nv, 8)
    ref = np.linalg.solve(A, v.reshape(2, -1).T).T.reshape(v.shape)
    x = torch.empty((2, pair.bl.V1, 2 * pair.Nv, 2), dtype=torch.float64, device="cuda")
    p = mglma.default_params(tol=1e-11, coarse=mglma.BF16, coarse_iters=16)
    pair.ctx.coarse_solve(to_dev(v), x, p)
    assert relerr(from_dev(x), ref) < 1e-9
    # pieces: D1^-1 R eta and W D2^-1 W^+ R eta
    eta = synth.gaussian_fields(2, pair.L, 9)
    Re = pair.B.restrict(pair.lat(eta)).reshape(2, -1)
    ge1_ref = np.linalg.solve(A, Re.T).T
    W = pair.top.W
    top_ref = (W @ np.linalg.solve(pair.top.D2, W.conj().T @ Re.T)).T
    ge1 = torch.empty_like(x)
    top = torch.empty_like(x)
    pair.ctx.coarse_pieces(pair.fine_dev(eta), ge1, top, p)
    assert relerr(from_dev(ge1).reshape(2, -1), ge1_ref) < 1e-9
    assert relerr(from_dev(top).reshape(2, -1), top_ref) < 1e-10


def test_error_paths(pair):
    from paper_2412_06347_amd import mglma
    b = synth.gaussian_fields(1, pair.L, 1)
    b[0, 3, 1, 2] = np.nan
    xd = pair.ctx.fine(1)
    rc, _ = pair.ctx.solve(pair.fine_dev(b), xd, mglma.default_params(), raise_on_error=False)
    assert rc == -4
    b = synth.gaussian_fields(1, pair.L, 2)
    rc, st = pair.ctx.solve(pair.fine_dev(b), xd, mglma.default_params(max_outer=1, max_inner=1),
                            raise_on_error=False)
    assert rc == -6 and st[0]["status"] == -6 and st[0]["true_rel_res"] > 1e-10
    # the CA-GCR smoother takes a Krylov dimension of at most 8
    rc, _ = pair.ctx.solve(pair.fine_dev(b), xd, mglma.default_params(smoother_alg=mglma.SMOOTH_CAGCR, nu_post=9),
                           raise_on_error=False)
    assert rc == -1
