"""The largest configuration's lattice on one GPU: 48^3 x 96 (V = 10,616,832
sites), 4^4 blocks.  The oracle cannot build the clover term of a lattice
this size in test time, so the gauge field is the seeded 48 x 24^3 field of
the benchmark tiled twice in every direction, with periodic fermion phases
in every direction (antiperiodic time would make a field tiled twice in
time periodic, not antiperiodic, over the large extent).  The operator then
commutes with translations by one tile and maps tiled fields to tiled
fields, which makes every full-size result checkable on one tile with the
oracle:

* the FP64 apply of a tiled field against the oracle's apply on one tile;
* the mixed-precision MG solve (block basis from tiled Gaussian test
  vectors, the benchmark's solver settings) of tiled right-hand sides: every
  tile of the solution equal, and one tile solving the small system to
  1e-10 under the oracle's operator (the residual of a tiled field is the
  tiled residual).
"""
import numpy as np
import pytest

from oracle import dirac
from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, from_dev, relerr

pytestmark = pytest.mark.gpu

LS = (48, 24, 24, 24)
LB = (96, 48, 48, 48)
B = (4, 4, 4, 4)
EPS, KAPPA, CSW, SEED = 0.25, 0.125, 1.0, 3
NV = 16
BC = (1.0, 1.0, 1.0, 1.0)


def _tile(f, L):
    """[n][V_small][...] canonical fields -> the same fields tiled 2x in every direction."""
    n, rest = f.shape[0], f.shape[2:]
    g = f.reshape(n, *L, *rest)
    g = np.tile(g, (1, 2, 2, 2, 2) + (1,) * len(rest))
    return g.reshape(n, -1, *rest)


def _tiles(f):
    """[n][V_big][4][3] -> [16][n][V_small][4][3], the 16 tiles in order."""
    n = f.shape[0]
    g = f.reshape(n, 2, LS[0], 2, LS[1], 2, LS[2], 2, LS[3], 4, 3)
    g = g.transpose(1, 3, 5, 7, 0, 2, 4, 6, 8, 9, 10)
    return g.reshape(16, n, -1, 4, 3)


@pytest.fixture(scope="module")
def big():
    import torch
    from paper_2412_06347_amd import mglma
    Us = synth.gauge_field(LS, EPS, SEED)
    D = dirac.WilsonClover(Us, LS, KAPPA, CSW, bc=BC)
    ctx = mglma.Context(LB, B, KAPPA, CSW, bc=BC)
    Ud = to_dev(_tile(Us[None], LS)[0])
    ctx.load_gauge(Ud)
    del Ud
    torch.cuda.synchronize()
    return ctx, D


def _export(ctx, dev):
    import torch
    out = torch.empty((dev.shape[0], ctx.V, 4, 3, 2), dtype=torch.float64, device="cuda")
    ctx.export_fields(dev, out)
    h = from_dev(out)
    del out
    return h


def test_maxsize_apply(big):
    ctx, D = big
    assert ctx.V == int(np.prod(LB))
    ps = synth.gaussian_fields(2, LS, 301)
    x = ctx.fine(2)
    ctx.import_fields(to_dev(_tile(ps, LS)), x)
    y = ctx.fine(2)
    ctx.apply_D(x, y)
    got = _tiles(_export(ctx, y))
    del x, y
    ref = dirac.fields_to_canonical(D.M(dirac.fields_to_lattice(ps, LS)))
    e = max(relerr(got[k], ref) for k in range(16))
    print("48^3x96 FP64 apply, largest tile error vs oracle: %.2e" % e)
    assert e < 1e-12


def test_maxsize_mg_solve(big):
    import torch
    import bench
    from paper_2412_06347_amd import mglma
    ctx, D = big
    tv = ctx.fine(NV)
    for c in range(NV):
        v = synth.gaussian_fields(1, LS, 400 + c)
        ctx.import_fields(to_dev(_tile(v, LS)), tv[c:c + 1])
    ctx.build_subspace(tv)
    del tv
    torch.cuda.empty_cache()
    assert ctx.V1 == int(np.prod(LB)) // 256 and ctx.nc == 2 * NV
    bs = synth.gaussian_fields(2, LS, 302)
    b = ctx.fine(2)
    ctx.import_fields(to_dev(_tile(bs, LS)), b)
    x = ctx.fine(2)
    rc, st = ctx.solve(b, x, bench.mixed_params(mglma, max_inner=400))
    print("48^3x96 MG solve: %d iterations, true rel res %s" % (st[0]["inner"], [s["true_rel_res"] for s in st]))
    assert rc == 0 and max(s["true_rel_res"] for s in st) <= 1e-10
    tiles = _tiles(_export(ctx, x))
    del b, x
    spread = max(relerr(tiles[k], tiles[0]) for k in range(1, 16))
    print("largest difference between tiles of the solution: %.2e" % spread)
    assert spread < 1e-12
    r = bs - dirac.fields_to_canonical(D.M(dirac.fields_to_lattice(tiles[0], LS)))
    res = (np.linalg.norm(r.reshape(2, -1), axis=1) / np.linalg.norm(bs.reshape(2, -1), axis=1)).max()
    print("one tile under the oracle's operator: relative residual %.2e" % res)
    assert res <= 1.05e-10
