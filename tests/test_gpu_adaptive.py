"""GPU checks of the adaptive (bootstrap) setup of the test vectors.  The
block basis is meant to span approximations of the low modes of Q (sec.
"Local coherence and block decomposition"); refining random test vectors by
inverse iteration with the current multigrid solver must lower the deficits
eq:cdeficit of the exact low modes (the oracle's dense eigenvectors of Q) and
the solver's iteration count.  The refined vectors are checked by
properties: each is normalised and, after one round, a multiple of it solves
M y = v_0 to the accuracy of the inner iterations under the oracle's
operator."""
import numpy as np
import pytest

from oracle import dirac
from paper_2412_06347_amd import synth
from tests.gpu_setup import Pair
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu

L, B, NV = (4, 4, 4, 4), (2, 2, 2, 2), 4


@pytest.fixture(scope="module")
def pair():
    return Pair(L, B, NV, kappa=0.124, oracle_galerkin=False)


def _params(mglma, **kw):
    return mglma.default_params(inner=mglma.F32, coarse=mglma.F32, gcr_m=16, **kw)


def _iterations(pair):
    from paper_2412_06347_amd import mglma
    b = synth.gaussian_fields(2, L, 91)
    x = pair.ctx.fine(2)
    rc, st = pair.ctx.solve(pair.fine_dev(b), x, _params(mglma, tol=1e-10, max_inner=400))
    assert rc == 0
    return max(s["inner"] for s in st)


def test_adaptive_one_round(pair):
    from paper_2412_06347_amd import mglma
    v0 = synth.gaussian_fields(NV, L, 92)
    tv = pair.fine_dev(v0)
    pair.ctx.build_subspace(tv)
    pair.ctx.adaptive_setup(tv, _params(mglma), rounds=1, iters=8)
    v1 = pair.fine_host(tv)
    assert np.abs(np.linalg.norm(v1.reshape(NV, -1), axis=1) - 1.0).max() < 1e-12
    Mv = pair.canon(pair.D.M(pair.lat(v1)))
    for c in range(NV):
        a, b = Mv[c].ravel(), v0[c].ravel()
        s = np.vdot(a, b) / np.vdot(a, a)
        res = np.linalg.norm(s * a - b) / np.linalg.norm(b)
        print("vector %d: |s M v_1 - v_0| / |v_0| = %.2e" % (c, res))
        assert res < 1e-2
    assert pair.ctx.nc == 2 * NV


def test_adaptive_improves_coherence(pair):
    from paper_2412_06347_amd import mglma
    lam, psi = dirac.low_modes(pair.D, 2 * NV)
    psid = pair.fine_dev(psi)
    tv = pair.fine_dev(synth.gaussian_fields(NV, L, 93))
    pair.ctx.build_subspace(tv)
    eps0, n0 = pair.ctx.deficit(psid), _iterations(pair)
    pair.ctx.adaptive_setup(tv, _params(mglma), rounds=3, iters=8)
    eps1, n1 = pair.ctx.deficit(psid), _iterations(pair)
    print("deficits of the %d lowest modes: random %s -> adaptive %s" % (2 * NV, np.round(eps0, 3),
                                                                      np.round(eps1, 3)))
    print("MG iterations to 1e-10: random %d -> adaptive %d" % (n0, n1))
    assert eps1.mean() < 0.8 * eps0.mean()
    assert n1 <= n0


def test_adaptive_arguments(pair):
    import torch
    from paper_2412_06347_amd import mglma
    tv = pair.fine_dev(synth.gaussian_fields(NV, L, 94))
    pair.ctx.build_subspace(tv)
    before = tv.clone()
    pair.ctx.adaptive_setup(tv, _params(mglma), rounds=0)       # no rounds: unchanged
    torch.cuda.synchronize()
    assert torch.equal(before, tv)
    for kw in (dict(rounds=-1), dict(iters=0)):
        with pytest.raises(mglma.MglmaError) as e:
            pair.ctx.adaptive_setup(tv, _params(mglma), **kw)
        assert e.value.code == -1
    # a context without a subspace: multigrid rounds need one, plain GCR rounds
    # (the bootstrap from nothing) build it
    ctx = mglma.Context(L, B, 0.124, 1.0)
    ctx.load_gauge(to_dev(pair.U))
    with pytest.raises(mglma.MglmaError) as e:
        ctx.adaptive_setup(tv, _params(mglma))
    assert e.value.code == -7
    ctx.adaptive_setup(tv, _params(mglma, use_mg=0), rounds=1, iters=8)
    assert ctx.nc == 2 * NV
